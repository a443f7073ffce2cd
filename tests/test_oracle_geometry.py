"""Pins of the aperture masks of §2.F: W_phi keeps the phase points that are a
corner of at least one valid subaperture (the geometry of the Shack-Hartmann
figure of §2.D: phase points on the subaperture corners)."""
import numpy as np

from oracle import geometry as G


def test_full_mask_keeps_every_phase_point():
    for n in (1, 2, 5, 10):
        m = G.valid_phase_mask(np.ones((n, n), bool))
        assert m.shape == (n + 1, n + 1)
        assert int(m.sum()) == (n + 1) ** 2


def test_ring_mask_counted_by_hand():
    # 4x4 subapertures, corners and the central 2x2 removed (8 valid).
    valid = np.array([[0, 1, 1, 0],
                      [1, 0, 0, 1],
                      [1, 0, 0, 1],
                      [0, 1, 1, 0]], bool)
    # corners of the 8 valid subapertures, listed row by row on the 5x5 points:
    # the centre point (2, 2) touches only the four removed central ones, and the
    # four outer corners (0,0), (0,4), (4,0), (4,4) only removed corner ones
    expect = np.array([[0, 1, 1, 1, 0],
                       [1, 1, 1, 1, 1],
                       [1, 1, 0, 1, 1],
                       [1, 1, 1, 1, 1],
                       [0, 1, 1, 1, 0]], bool)
    m = G.valid_phase_mask(valid)
    assert np.array_equal(m, expect)
    assert int(m.sum()) == 20


def test_single_subaperture_has_four_corners():
    for i, j in ((0, 0), (2, 1), (3, 3)):
        valid = np.zeros((4, 4), bool)
        valid[i, j] = True
        m = G.valid_phase_mask(valid)
        assert sorted(zip(*np.nonzero(m))) == [(i, j), (i, j + 1), (i + 1, j), (i + 1, j + 1)]


def test_phase_points_are_subaperture_corners():
    n, d = 3, 0.7
    c = G.subap_centers(n, d)
    p = G.phase_points(n, d).reshape(n + 1, n + 1, 2)
    for k in range(n * n):
        i, j = divmod(k, n)
        corners = np.array([p[i, j], p[i, j + 1], p[i + 1, j], p[i + 1, j + 1]])
        assert np.allclose(corners.mean(axis=0), c[k])
        assert np.allclose(np.abs(corners - c[k]), d / 2)
