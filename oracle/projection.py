"""Second step phi_beta = W_phi Sigma_{phi_beta s} zeta (§2.C, §2.F), in float64.

For LGS the phase-slope covariance is not 2RBT because the target phase and
the slopes are sampled differently (§2.D, cone effect).  §2.D replaces, for
every layer k, the target phase by a new grid phi'_k of spacing d_k = s_k d
(the slope sampling of that layer); Xi'_{q,k} = <phi'_k s_q^T> is then 2RBT,
and the target phase on the original grid is recovered by bilinear
interpolation I'_k:  Xi_q = sum_k I'_k Xi'_{q,k}.  §2.E uses one common grid
size n' (the one the highest layer needs) for all layers so that a single
shuffle S1 and a single set of forward transforms serve every layer.

Readings (the paper fixes neither the size formula nor the centring):
  * n' = ceil(n / min_k s_k) + 1, so the n' x n' grid of spacing s_k d covers
    the (n+1) x (n+1) phase points for every layer;
  * every grid is centred on the reconstruction direction:
    rho'_{i'j'} = ((j' - (n'-1)/2) s_k d, (i' - (n'-1)/2) s_k d) in pupil
    coordinates, seen along the target direction beta at altitude h_k;
  * I'_k is the standard bilinear interpolation from that grid to the phase
    points; grid nodes outside the grid contribute zero (never needed with the
    n' above).
With natural guide stars (s_k = 1) and n' = n + 1 the grid coincides with the
phase points, I'_k is the identity and the result is the exact product.

Functions:
  phi_paper_dense  dense Xi'_{q,k} and I'_k, summed over layers (definition)
  phi_paper_fft    the same through the §2.E LGS equation: forward transforms of
                   S1 zeta_q once, per-layer products summed over q, one
                   inverse transform per layer, then I'_k S2
  phi_exact        W_phi Sigma_{phi_beta s} zeta with the exact covariance, for
                   reporting the interpolation gap only
"""
import math

import numpy as np

from . import geometry as G
from .covariance import phase_fns, phase_slope_cov


def new_grid_size(wl):
    s = G.cone_scale(wl.h, wl.h_lgs)
    return int(math.ceil(wl.n / float(np.min(s)) - 1e-12)) + 1


def grid_points(wl, k, n_prime):
    """(n'^2, 2) coordinates of the layer-k grid, index i'*n' + j'."""
    s = G.cone_scale(wl.h, wl.h_lgs)[k]
    i, j = np.divmod(np.arange(n_prime * n_prime), n_prime)
    c = (n_prime - 1) / 2.0
    return np.stack([(j - c) * s * wl.d, (i - c) * s * wl.d], axis=1)


def xi_prime(wl, k, n_prime, beta=None):
    """Dense Xi'_{.,k}: (n'^2, n_slopes) covariance of the layer-k grid phase
    (along the target direction) with every valid slope (App. A.2 phase-slope
    model, layer k only, weight w_k)."""
    beta = np.asarray(wl.target if beta is None else beta, dtype=np.float64)
    s = G.cone_scale(wl.h, wl.h_lgs)[k]
    rho = grid_points(wl, k, n_prime)
    r = G.subap_centers(wl.n, wl.d)[G.valid_index(wl.valid)]
    nv = r.shape[0]
    out = np.zeros((rho.shape[0], 2 * wl.n_gs * nv))
    fx, fy = phase_fns(wl)
    for g in range(wl.n_gs):
        ox = s * r[None, :, 0] + wl.h[k] * (wl.gs[g, 0] - beta[0]) - rho[:, None, 0]
        oy = s * r[None, :, 1] + wl.h[k] * (wl.gs[g, 1] - beta[1]) - rho[:, None, 1]
        out[:, 2 * g * nv:(2 * g + 1) * nv] = wl.w[k] * fx(ox, oy, s * wl.d, wl.r0, wl.L0)
        out[:, (2 * g + 1) * nv:(2 * g + 2) * nv] = wl.w[k] * fy(ox, oy, s * wl.d, wl.r0, wl.L0)
    return out


def interp_matrix(wl, k, n_prime):
    """Dense I'_k: ((n+1)^2, n'^2) bilinear interpolation from the layer-k grid
    to the phase points."""
    s = G.cone_scale(wl.h, wl.h_lgs)[k]
    rho = G.phase_points(wl.n, wl.d)
    c = (n_prime - 1) / 2.0
    I = np.zeros((rho.shape[0], n_prime * n_prime))
    fx = rho[:, 0] / (s * wl.d) + c
    fy = rho[:, 1] / (s * wl.d) + c
    for m in range(rho.shape[0]):
        j0 = int(math.floor(fx[m]))
        i0 = int(math.floor(fy[m]))
        tx = fx[m] - j0
        ty = fy[m] - i0
        for di, dj, wgt in ((0, 0, (1 - tx) * (1 - ty)), (0, 1, tx * (1 - ty)),
                            (1, 0, (1 - tx) * ty), (1, 1, tx * ty)):
            ii, jj = i0 + di, j0 + dj
            if 0 <= ii < n_prime and 0 <= jj < n_prime and wgt != 0.0:
                I[m, ii * n_prime + jj] += wgt
    return I


def phi_paper_dense(wl, zeta, n_prime=None):
    """W_phi sum_k I'_k Xi'_{.,k} zeta (definition of §2.D)."""
    n_prime = new_grid_size(wl) if n_prime is None else n_prime
    phi = np.zeros((wl.n + 1) ** 2)
    for k in range(wl.n_layer):
        phi += interp_matrix(wl, k, n_prime) @ (xi_prime(wl, k, n_prime) @ zeta)
    return phi[G.valid_phase_mask(wl.valid).ravel()]


def xi_prime_table(wl, k, g, p, n_prime, beta=None):
    """Unique elements of the 2RBT block Xi'_{q,k} (q = (g, p)): array
    t[v + n'-1, u + n'-1] for lags u, v in [-(n'-1), n-1] (subaperture index minus
    grid index), (n'+n-1)^2 values (§2.D)."""
    beta = np.asarray(wl.target if beta is None else beta, dtype=np.float64)
    s = G.cone_scale(wl.h, wl.h_lgs)[k]
    off = (n_prime - wl.n) / 2.0
    lag = np.arange(-(n_prime - 1), wl.n)
    U, V = np.meshgrid(lag, lag)
    ox = s * wl.d * (U + off) + wl.h[k] * (wl.gs[g, 0] - beta[0])
    oy = s * wl.d * (V + off) + wl.h[k] * (wl.gs[g, 1] - beta[1])
    f = phase_fns(wl)[p]
    return wl.w[k] * f(ox, oy, s * wl.d, wl.r0, wl.L0)


def _xi_job(args):
    wl, k, q, n_prime = args
    return (k, q), xi_prime_table(wl, k, q // 2, q % 2, n_prime)


def xi_prime_tables(wl, n_prime=None, workers=1):
    """dict (k, q) -> unique elements of every Xi'_{q,k}; workers > 1 uses a process pool."""
    n_prime = new_grid_size(wl) if n_prime is None else n_prime
    jobs = [(wl, k, q, n_prime) for k in range(wl.n_layer) for q in range(2 * wl.n_gs)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            return dict(pool.map(_xi_job, jobs, chunksize=4))
    return dict(_xi_job(j) for j in jobs)


def default_proj_pad(n, n_prime):
    m = n_prime + n - 1
    return m + (m & 1)


def phi_paper_fft(wl, zeta, n_prime=None, L=None, tables=None):
    """§2.E LGS equation with common n': one S1 and one forward FFT per channel,
    per layer the products summed over channels, one inverse FFT, then I'_k S2."""
    n, C = wl.n, 2 * wl.n_gs
    n_prime = new_grid_size(wl) if n_prime is None else n_prime
    L = default_proj_pad(n, n_prime) if L is None else L
    if L < n_prime + n - 1:
        raise ValueError("L must be >= n' + n - 1")
    nv = wl.n_vs
    z = np.asarray(zeta, dtype=np.float64).reshape(C, nv)
    idx = G.valid_index(wl.valid)
    zt = []
    for q in range(C):                                   # S1, forward FFT, once
        b = np.zeros((L, L))
        full = np.zeros(n * n)
        full[idx] = z[q]
        b[:n, :n] = full.reshape(n, n)
        zt.append(np.fft.rfft2(b))
    lag = np.arange(-(n_prime - 1), n)
    pos = (-lag) % L
    phi = np.zeros((n + 1) ** 2)
    for k in range(wl.n_layer):
        acc = np.zeros_like(zt[0])
        for q in range(C):
            t = (tables[(k, q)] if tables is not None
                 else xi_prime_table(wl, k, q // 2, q % 2, n_prime))
            K = np.zeros((L, L))
            K[np.ix_(pos, pos)] = t
            acc += np.fft.rfft2(K) * zt[q]               # element-wise products, summed
        c = np.fft.irfft2(acc, s=(L, L))                 # one inverse per layer
        phik = c[:n_prime, :n_prime].ravel()             # S2
        phi += interp_matrix(wl, k, n_prime) @ phik      # I'_k
    return phi[G.valid_phase_mask(wl.valid).ravel()]


def phi_exact(wl, zeta):
    """W_phi Sigma_{phi_beta s} zeta with the exact Hudgin phase-slope covariance."""
    rho = G.phase_points(wl.n, wl.d)[G.valid_phase_mask(wl.valid).ravel()]
    return phase_slope_cov(wl, rho) @ zeta
