"""Hudgin-like covariance model, dense matrices (App. A.2; §2.C-§2.F).

A Hudgin-like slope is the phase difference between the two edge midpoints of
a subaperture (App. A.2); a Fried slope (App. A.3, selected by a workload
attribute model = 'fried') is half the sum of the two corner-to-corner
differences across the subaperture.  With the structure function D of the von Karman
model, the slope-slope covariances of one layer at separation Delta and edge
spacing delta are (App. A.2, Hudgin slope-slope equations):

  xx(Delta) = 1/2 [ -2 D(Delta) + D(Delta + delta x) + D(Delta - delta x) ]
  yy(Delta) = the same with y
  xy(Delta) = yx(Delta) = 1/2 [ D(Delta + delta(x+y)/2) - D(Delta + delta(-x+y)/2)
                                - D(Delta + delta(x-y)/2) + D(Delta - delta(x+y)/2) ]

Reading: the printed xy formula ends with "- D(Delta - dx/2 - dy/2)"; expanding
the product of the two phase differences with the identity printed in App. A.2
gives "+", which is also the only sign for which xy(0) = 0 (isotropy).  The
factor (lambda / 2 pi d)^2 of the printed formulas is dropped: slopes are phase
differences in radians.

Layers add, D_k = w_k D (D scales as r0^(-5/3)).  For guide stars i, j and a
slope of sensor i at subaperture a and a slope of sensor j at b, layer k sees
(§2.D cone effect, LGS at h_lgs):

  Delta_k = s_k (r_b - r_a) + h_k (alpha_j - alpha_i),   delta_k = s_k d,

s_k = 1 - h_k / h_lgs.  Both the separation and the edge spacing shrink with
the cone; the guide-star baseline does not.  For natural guide stars s_k = 1.

The phase-slope covariance of a target phase point rho (target at infinity,
on-axis by default) and a slope of sensor j at b is (App. A.2, Hudgin
phase-slope equation, without the lambda/(4 pi d) factor and with the
second 'replacing dx' read as giving the y component):

  phi-x(Delta) = 1/2 [ D(Delta - delta x/2) - D(Delta + delta x/2) ],
  Delta = s_k r_b + h_k alpha_j - (rho + h_k beta),  delta = s_k d.
"""
import numpy as np

from . import geometry as G
from .vonkarman import structure_function


def _D(dx, dy, r0, L0):
    return structure_function(np.hypot(dx, dy), r0, L0)


def hudgin_xx(dx, dy, delta, r0, L0):
    return 0.5 * (-2.0 * _D(dx, dy, r0, L0) + _D(dx + delta, dy, r0, L0) + _D(dx - delta, dy, r0, L0))


def hudgin_yy(dx, dy, delta, r0, L0):
    return 0.5 * (-2.0 * _D(dx, dy, r0, L0) + _D(dx, dy + delta, r0, L0) + _D(dx, dy - delta, r0, L0))


def hudgin_xy(dx, dy, delta, r0, L0):
    h = 0.5 * delta
    return 0.5 * (_D(dx + h, dy + h, r0, L0) - _D(dx - h, dy + h, r0, L0)
                  - _D(dx + h, dy - h, r0, L0) + _D(dx - h, dy - h, r0, L0))


def fried_xx(dx, dy, delta, r0, L0):
    """App. A.3 Fried slope-slope xx: 1/8 [-4 D + 2 F1 - 2 F2 + F3 + F4] (slopes in rad:
    the printed 1/2 (lambda / 4 pi d)^2 is (lambda / 2 pi d)^2 / 8)."""
    F1, F2, F3, F4 = _fried_F(dx, dy, delta, r0, L0)
    return 0.125 * (-4.0 * _D(dx, dy, r0, L0) + 2.0 * F1 - 2.0 * F2 + F3 + F4)


def fried_yy(dx, dy, delta, r0, L0):
    F1, F2, F3, F4 = _fried_F(dx, dy, delta, r0, L0)
    return 0.125 * (-4.0 * _D(dx, dy, r0, L0) - 2.0 * F1 + 2.0 * F2 + F3 + F4)


def fried_xy(dx, dy, delta, r0, L0):
    F1, F2, F3, F4 = _fried_F(dx, dy, delta, r0, L0)
    return 0.125 * (F3 - F4)


def _fried_F(dx, dy, delta, r0, L0):
    F1 = _D(dx + delta, dy, r0, L0) + _D(dx - delta, dy, r0, L0)
    F2 = _D(dx, dy + delta, r0, L0) + _D(dx, dy - delta, r0, L0)
    F3 = _D(dx + delta, dy + delta, r0, L0) + _D(dx - delta, dy - delta, r0, L0)
    F4 = _D(dx + delta, dy - delta, r0, L0) + _D(dx - delta, dy + delta, r0, L0)
    return F1, F2, F3, F4


def fried_phase_x(dx, dy, delta, r0, L0):
    """App. A.3 Fried phase-slope x: 1/4 (-F5 + F6 + F7 - F8) in rad (printed lambda/(8 pi d))."""
    h = 0.5 * delta
    F5, F6 = _D(dx + h, dy + h, r0, L0), _D(dx - h, dy + h, r0, L0)
    F7, F8 = _D(dx - h, dy - h, r0, L0), _D(dx + h, dy - h, r0, L0)
    return 0.25 * (-F5 + F6 + F7 - F8)


def fried_phase_y(dx, dy, delta, r0, L0):
    h = 0.5 * delta
    F5, F6 = _D(dx + h, dy + h, r0, L0), _D(dx - h, dy + h, r0, L0)
    F7, F8 = _D(dx - h, dy - h, r0, L0), _D(dx + h, dy - h, r0, L0)
    return 0.25 * (-F5 - F6 + F7 + F8)


def hudgin_phase_x(dx, dy, delta, r0, L0):
    return 0.5 * (_D(dx - 0.5 * delta, dy, r0, L0) - _D(dx + 0.5 * delta, dy, r0, L0))


def hudgin_phase_y(dx, dy, delta, r0, L0):
    return 0.5 * (_D(dx, dy - 0.5 * delta, r0, L0) - _D(dx, dy + 0.5 * delta, r0, L0))


_SS = {(0, 0): hudgin_xx, (1, 1): hudgin_yy, (0, 1): hudgin_xy, (1, 0): hudgin_xy}
_SS_FRIED = {(0, 0): fried_xx, (1, 1): fried_yy, (0, 1): fried_xy, (1, 0): fried_xy}


def model_of(wl):
    """Gradient model of a workload: 'hudgin' (App. A.2, default) or 'fried' (App. A.3)."""
    return getattr(wl, "model", "hudgin")


def phase_fns(wl):
    return (fried_phase_x, fried_phase_y) if model_of(wl) == "fried" else (hudgin_phase_x, hudgin_phase_y)


def slope_pair_cov(wl, gi, p, ra, gj, q, rb):
    """Covariance of slope component p of sensor gi at subaperture centres ra (m, 2)
    with slope component q of sensor gj at centres rb (m, 2), element-wise,
    summed over layers (App. A.2 with the §2.D cone scaling)."""
    s = G.cone_scale(wl.h, wl.h_lgs)
    f = (_SS_FRIED if model_of(wl) == "fried" else _SS)[(p, q)]
    out = np.zeros(np.broadcast_shapes(ra.shape[:-1], rb.shape[:-1]))
    for k in range(wl.n_layer):
        base = wl.h[k] * (wl.gs[gj] - wl.gs[gi])
        dx = s[k] * (rb[..., 0] - ra[..., 0]) + base[0]
        dy = s[k] * (rb[..., 1] - ra[..., 1]) + base[1]
        out = out + wl.w[k] * f(dx, dy, s[k] * wl.d, wl.r0, wl.L0)
    return out


def slope_covariance(wl):
    """Dense Sigma_ss restricted to valid slopes, W_s Sigma_ss W_s^T (§2.D, §2.F),
    ordered as in geometry's slope layout.  Entry by entry from the positions."""
    r = G.subap_centers(wl.n, wl.d)[G.valid_index(wl.valid)]
    nv = r.shape[0]
    C = 2 * wl.n_gs
    S = np.zeros((C * nv, C * nv))
    ra = r[:, None, :]
    rb = r[None, :, :]
    for a in range(C):
        for b in range(a, C):
            blk = slope_pair_cov(wl, a // 2, a % 2, ra, b // 2, b % 2, rb)
            S[a * nv:(a + 1) * nv, b * nv:(b + 1) * nv] = blk
            if b != a:
                S[b * nv:(b + 1) * nv, a * nv:(a + 1) * nv] = blk.T
    return S


def noise_covariance(wl, noise_var=None, noise_xy=None):
    """Sigma_eta on the valid slopes (§2.C; §2.F elongated LGS spots): the
    per-slope variances on the diagonal (a scalar sigma^2 or one per slope),
    and with noise_xy (n_gs, n_vs) the x-y covariance of each subaperture in
    each sensor, which makes Sigma_eta 2x2 block diagonal."""
    nv = wl.noise_var if noise_var is None else noise_var
    N = wl.n_slopes
    E = np.diag(np.broadcast_to(np.asarray(nv, dtype=np.float64), (N,)).copy())
    if noise_xy is not None:
        nvs = N // (2 * wl.n_gs)
        for g in range(wl.n_gs):
            for v in range(nvs):
                i, j = 2 * g * nvs + v, (2 * g + 1) * nvs + v
                E[i, j] = E[j, i] = noise_xy[g, v]
    return E


def system_matrix(wl, noise_var=None, noise_xy=None):
    """A = W_s (Sigma_ss + Sigma_eta) W_s^T (§2.C, §2.F)."""
    return slope_covariance(wl) + noise_covariance(wl, noise_var, noise_xy)


def slope_covariance_rows(wl, rows):
    """Selected rows of W_s Sigma_ss W_s^T (global slope indices), entry by entry."""
    r = G.subap_centers(wl.n, wl.d)[G.valid_index(wl.valid)]
    nv = r.shape[0]
    C = 2 * wl.n_gs
    rows = np.asarray(rows)
    out = np.zeros((rows.size, C * nv))
    for t, row in enumerate(rows):
        a, va = divmod(int(row), nv)
        for b in range(C):
            out[t, b * nv:(b + 1) * nv] = slope_pair_cov(wl, a // 2, a % 2, r[va][None, :], b // 2, b % 2, r)
    return out


def kernel_table(wl, gi, gj, p, q):
    """Unique elements of the 2RBT block Theta^{gi gj}_{pq} (§2.D): the
    (2n-1) x (2n-1) array t[v + n-1, u + n-1] = covariance at subaperture lag
    (u, v) = (column, row) offset of the second slope relative to the first,
    so that Theta[a, b] = t(lag(b) - lag(a))."""
    n = wl.n
    lag = np.arange(-(n - 1), n) * wl.d
    U, V = np.meshgrid(lag, lag)
    rb = np.stack([U, V], axis=-1)
    ra = np.zeros_like(rb)
    return slope_pair_cov(wl, gi, p, ra, gj, q, rb)


def _table_job(args):
    wl, a, b = args
    return (a, b, kernel_table(wl, a // 2, b // 2, a % 2, b % 2))


def kernel_tables(wl, workers=1):
    """All unique blocks: dict (gi, gj, p, q) -> (2n-1, 2n-1) for every ordered
    channel pair.  Channel pairs a <= b (a = 2 gi + p) are evaluated; the others
    follow from the symmetry of a covariance, Theta^{ji}_{qp}(lag) =
    Theta^{ij}_{pq}(-lag), i.e. the table reversed along both axes.
    workers > 1 evaluates the tables in a process pool."""
    C = 2 * wl.n_gs
    jobs = [(wl, a, b) for a in range(C) for b in range(a, C)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_table_job, jobs, chunksize=1)
    else:
        res = [_table_job(j) for j in jobs]
    out = {}
    for a, b, t in res:
        out[(a // 2, b // 2, a % 2, b % 2)] = t
        if a != b:
            out[(b // 2, a // 2, b % 2, a % 2)] = t[::-1, ::-1].copy()
    return out


def phase_slope_cov(wl, rho, target=None):
    """Exact Sigma_{phi_beta s}: covariance of the target phase at points rho (m, 2)
    with every valid slope (m, C*n_vs) (App. A.2 phase-slope model, §2.C).
    The target is at infinity in direction beta (default wl.target)."""
    beta = np.asarray(wl.target if target is None else target, dtype=np.float64)
    r = G.subap_centers(wl.n, wl.d)[G.valid_index(wl.valid)]
    nv = r.shape[0]
    s = G.cone_scale(wl.h, wl.h_lgs)
    out = np.zeros((rho.shape[0], 2 * wl.n_gs * nv))
    fx, fy = phase_fns(wl)
    for g in range(wl.n_gs):
        for k in range(wl.n_layer):
            ox = s[k] * r[None, :, 0] + wl.h[k] * (wl.gs[g, 0] - beta[0]) - rho[:, None, 0]
            oy = s[k] * r[None, :, 1] + wl.h[k] * (wl.gs[g, 1] - beta[1]) - rho[:, None, 1]
            dl = s[k] * wl.d
            out[:, (2 * g) * nv:(2 * g + 1) * nv] += wl.w[k] * fx(ox, oy, dl, wl.r0, wl.L0)
            out[:, (2 * g + 1) * nv:(2 * g + 2) * nv] += wl.w[k] * fy(ox, oy, dl, wl.r0, wl.L0)
    return out
