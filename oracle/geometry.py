"""Sensor geometry (§2 and §2.D: n x n subapertures, (n+1) x (n+1) phase points;
§2.D "Slope-Slope Covariance Matrix": LGS cone effect; §2.F: aperture masks).

Conventions: subaperture (i, j) is row i (y) and column j (x), flattened
k = i*n + j (the index rule of §2.E step 1).  Subaperture centres are
((j - (n-1)/2) d, (i - (n-1)/2) d); phase points sit on subaperture corners
((j - n/2) d, (i - n/2) d), 0 <= i, j <= n.  A phase point is valid when it is a
corner of at least one valid subaperture.

Slope vector layout (the concatenation of §2, sensor by sensor, each sensor's
x slopes then y slopes, restricted by W_s to valid subapertures in row-major
order): channel c = 2*g + p (g = guide star, p = 0 for x, 1 for y), entry
c*n_vs + v.
"""
import math

import numpy as np


def subap_centers(n, d):
    """(n*n, 2) centres r_k = (x, y) of all subapertures, k = i*n + j."""
    i, j = np.divmod(np.arange(n * n), n)
    return np.stack([(j - (n - 1) / 2.0) * d, (i - (n - 1) / 2.0) * d], axis=1)


def phase_points(n, d):
    """((n+1)^2, 2) phase-point coordinates, index i*(n+1) + j."""
    i, j = np.divmod(np.arange((n + 1) * (n + 1)), n + 1)
    return np.stack([(j - n / 2.0) * d, (i - n / 2.0) * d], axis=1)


def valid_phase_mask(valid):
    """(n+1, n+1) bool: corners of valid subapertures (W_phi of §2.F)."""
    n = valid.shape[0]
    m = np.zeros((n + 1, n + 1), dtype=bool)
    m[:-1, :-1] |= valid
    m[:-1, 1:] |= valid
    m[1:, :-1] |= valid
    m[1:, 1:] |= valid
    return m


def cone_scale(h, h_lgs):
    """Cone factor s_k = 1 - h_k / h_lgs of the LGS footprint at altitude h_k
    (the sampling d_k = d (h_lgs - h_k) / h_lgs of §2.D); 1 for a natural
    guide star (h_lgs = inf)."""
    h = np.asarray(h, dtype=np.float64)
    if math.isinf(h_lgs):
        return np.ones_like(h)
    return 1.0 - h / h_lgs


def valid_index(valid):
    """Row-major indices k = i*n + j of the valid subapertures."""
    return np.flatnonzero(np.asarray(valid).ravel())
