"""Pins of the second step (§2.C), the LGS per-layer grid + bilinear form of
§2.D and its FFT evaluation (§2.E LGS equation)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import projection as P
from oracle.vonkarman import structure_function


def independent_phase_slope(wl, rho):
    """cov(phi_beta(rho), phi(P) - phi(Q)) from point covariances sigma^2 - D/2."""
    idx = G.valid_index(wl.valid)
    r = G.subap_centers(wl.n, wl.d)[idx]
    s = G.cone_scale(wl.h, wl.h_lgs)
    out = np.zeros((rho.shape[0], wl.n_slopes))
    cov = lambda a, b: 3.0 - 0.5 * structure_function(np.hypot(*(a - b).T), wl.r0, wl.L0)
    col = 0
    for g in range(wl.n_gs):
        for p in range(2):
            e = np.array([1.0, 0.0]) if p == 0 else np.array([0.0, 1.0])
            for v in range(r.shape[0]):
                for k in range(wl.n_layer):
                    c = s[k] * r[v] + wl.h[k] * wl.gs[g]
                    Pp = c + 0.5 * s[k] * wl.d * e
                    Qp = c - 0.5 * s[k] * wl.d * e
                    tgt = rho + wl.h[k] * np.asarray(wl.target)
                    out[:, col] += wl.w[k] * (cov(tgt, Pp[None]) - cov(tgt, Qp[None]))
                col += 1
    return out


def test_exact_phase_slope_matches_point_covariances():
    wl = W.tiny(n=3, n_gs=2, lgs=True, n_layer=2, seed=4)
    rho = G.phase_points(wl.n, wl.d)
    from oracle.covariance import phase_slope_cov
    A = phase_slope_cov(wl, rho)
    B = independent_phase_slope(wl, rho)
    assert np.abs(A - B).max() <= 1e-11 * np.abs(B).max()


@pytest.mark.parametrize("target", [(0.0, 0.0), (5e-5, -3e-5)])
def test_ngs_grid_is_identity_and_exact(target):
    wl = W.tiny(n=4, n_gs=3, lgs=False, n_layer=3, seed=6)
    wl.target = target
    assert P.new_grid_size(wl) == wl.n + 1
    for k in range(wl.n_layer):
        assert np.abs(P.interp_matrix(wl, k, wl.n + 1) - np.eye((wl.n + 1) ** 2)).max() < 1e-12
    z = np.random.default_rng(0).standard_normal(wl.n_slopes)
    a = P.phi_paper_dense(wl, z)
    e = P.phi_exact(wl, z)
    assert np.abs(a - e).max() <= 1e-11 * np.abs(e).max()


def test_bilinear_reproduces_affine_functions():
    wl = W.tiny(n=5, n_gs=2, lgs=True, n_layer=3, seed=2)
    n_prime = P.new_grid_size(wl)
    for k in range(wl.n_layer):
        I = P.interp_matrix(wl, k, n_prime)
        g = P.grid_points(wl, k, n_prime)
        f = lambda q: 0.3 + 1.7 * q[:, 0] - 0.9 * q[:, 1]
        rho = G.phase_points(wl.n, wl.d)
        assert np.abs(I @ f(g) - f(rho)).max() < 1e-12
        assert np.allclose(I.sum(axis=1), 1.0)


@pytest.mark.parametrize("n,g,seed", [(3, 1, 0), (4, 2, 1), (5, 3, 2), (6, 2, 3)])
def test_fft_form_equals_dense_form(n, g, seed):
    wl = W.tiny(n=n, n_gs=g, lgs=True, n_layer=3, seed=seed)
    z = np.random.default_rng(seed).standard_normal(wl.n_slopes)
    a = P.phi_paper_dense(wl, z)
    n_prime = P.new_grid_size(wl)
    for L in (n_prime + n - 1, n_prime + n + 2):
        b = P.phi_paper_fft(wl, z, L=L)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_interpolation_gap_is_small_for_config1():
    wl = W.lgs3_10x10()
    z = np.random.default_rng(5).standard_normal(wl.n_slopes)
    a = P.phi_paper_dense(wl, z)
    e = P.phi_exact(wl, z)
    gap = np.linalg.norm(a - e) / np.linalg.norm(e)
    assert 1e-6 < gap < 0.2


def test_grid_size_config2():
    assert P.new_grid_size(W.lgs6_74x74()) == 106
    assert P.new_grid_size(W.lgs3_10x10()) == 13


def test_fried_phase_slope_matches_corner_points():
    wl = W.tiny(n=3, n_gs=2, lgs=True, n_layer=2, seed=4)
    wl.model = "fried"
    rho = G.phase_points(wl.n, wl.d)
    from oracle.covariance import phase_slope_cov
    A = phase_slope_cov(wl, rho)
    idx = G.valid_index(wl.valid)
    r = G.subap_centers(wl.n, wl.d)[idx]
    s = G.cone_scale(wl.h, wl.h_lgs)
    cov = lambda a, b: 2.0 - 0.5 * structure_function(np.hypot(*(a - b).T), wl.r0, wl.L0)
    corners = np.array([[1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=float)
    wts = {0: [0.5, -0.5, -0.5, 0.5], 1: [0.5, 0.5, -0.5, -0.5]}
    B = np.zeros_like(A)
    col = 0
    for g in range(wl.n_gs):
        for p in range(2):
            for v in range(r.shape[0]):
                for k in range(wl.n_layer):
                    c0 = s[k] * r[v] + wl.h[k] * wl.gs[g]
                    for q in range(4):
                        B[:, col] += wl.w[k] * wts[p][q] * cov(rho, (c0 + 0.5 * s[k] * wl.d * corners[q])[None])
                col += 1
    assert np.abs(A - B).max() <= 1e-11 * np.abs(B).max()


@pytest.mark.parametrize("n,target", [(4, (0.0, 0.0)), (6, (0.0, 0.0)), (4, (4e-5, -2e-5))])
def test_lgs_grid_nodes_on_phase_points_give_the_exact_product(n, target):
    """Layers at h = 0 and h = H/2 (s_k = 1 and 1/2) with n even: the common grid
    of §2.D (n' = 2n + 1 nodes of spacing s_k d, centred on the target ray)
    holds every phase point as a node, so the bilinear I'_k only selects nodes
    and the paper's form equals the exact W_phi Sigma_phi_s zeta.  A slip in
    the grid size, its centring or the node spacing moves the phase points off
    the nodes and breaks the equality."""
    wl = W.tiny(n=n, n_gs=3, lgs=True, n_layer=2, seed=11, mask="random")
    wl.h = np.array([0.0, 0.5 * wl.h_lgs])
    wl.target = target
    assert np.allclose(G.cone_scale(wl.h, wl.h_lgs), [1.0, 0.5])
    n_prime = P.new_grid_size(wl)
    assert n_prime == 2 * n + 1
    for k in range(wl.n_layer):
        I = P.interp_matrix(wl, k, n_prime)
        assert set(np.unique(np.round(I, 12))) <= {0.0, 1.0}
        assert np.all(np.count_nonzero(np.abs(I) > 1e-12, axis=1) == 1)
    z = np.random.default_rng(n).standard_normal(wl.n_slopes)
    e = P.phi_exact(wl, z)
    a = P.phi_paper_dense(wl, z)
    b = P.phi_paper_fft(wl, z)
    assert np.abs(a - e).max() <= 1e-12 * np.abs(e).max()
    assert np.abs(b - e).max() <= 1e-12 * np.abs(e).max()
