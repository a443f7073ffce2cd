"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module only describes inputs: telescope and wave-front-sensor geometry,
guide-star directions, a layered turbulence profile, the noise level and
measured slope vectors drawn from simulated turbulence.  It contains none of
the reconstructor's arithmetic (no covariances, no Toeplitz products, no
solver) and imports neither the oracle nor the HIP library.

Workloads (parameters follow Table 1 and Table 2 of the paper where they exist,
with the readings listed in each constructor):

  lgs3_10x10  8 m pupil, 30 % obstruction, 10x10 Shack-Hartmann, 3 LGS at 90 km on a
      30 arcsec ring, layers 0 / 10 km (0.7 / 0.3), r0 = 0.15 m, L0 = 25 m,
      sigma^2 = 0.1 rad^2, FFT side L = 20.  76 valid subapertures, 456 slopes.
  lgs6_74x74  39 m pupil, 28 % obstruction, 74x74, 6 LGS at 90 km on a 60 arcsec ring,
      35 layers 30 m - 26.5 km with seeded exponentially decaying weights,
      r0 = 0.157 m, L0 = 25 m, sigma^2 = 0.1 rad^2, L = 148.  3972 valid
      subapertures per sensor, 47 664 slopes.  Stands in for the HARMONI LTAO
      system of Table 2, whose 35-layer profile is only given as a figure.
  lgs6_74x74_family(i)  the 74x74 geometry with seeded layer weights and r0 in
      [0.10, 0.25] m: distinct systems for batched products (L = 256 by default).
  uneven_family(i)  uneven systems (grids 40 / 60 / 74 / 84, 4-8 LGS, 10-35
      layers, noise 0.01-0.5 rad^2) for batched solves of different systems.
  tiny(...)  small seeded variants (n = 2..8, 1-4 guide stars, NGS or LGS)
             used for exhaustive CPU checks.

Units: angles in radians, lengths in metres, phase in radians at 500 nm.
Slopes are phase differences across one subaperture (rad), so that the noise
variance sigma^2 is comparable with the slope variance.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

ARCSEC = math.pi / 648000.0
SEED = 1806


@dataclasses.dataclass
class Workload:
    name: str
    n: int                      # subapertures across one sensor
    D: float                    # pupil diameter [m]
    obstruction: float          # central obstruction, diameter ratio
    gs: np.ndarray              # (n_gs, 2) guide-star directions [rad] (x, y)
    h_lgs: float                # LGS altitude [m]; math.inf for natural guide stars
    h: np.ndarray               # (n_layer,) layer altitudes [m]
    w: np.ndarray               # (n_layer,) fractional C_n^2 weights, sum 1
    r0: float                   # Fried parameter at 500 nm [m]
    L0: float                   # outer scale [m]
    noise_var: float            # slope noise variance [rad^2]
    pad_L: int                  # FFT side for the slope-slope products
    valid: np.ndarray           # (n, n) bool, row-major, row i = y, column j = x
    target: tuple = (0.0, 0.0)  # reconstruction direction [rad]
    model: str = "hudgin"       # gradient model of the reconstructor: "hudgin" or "fried"

    @property
    def d(self) -> float:
        return self.D / self.n

    @property
    def n_gs(self) -> int:
        return int(self.gs.shape[0])

    @property
    def n_layer(self) -> int:
        return int(self.h.shape[0])

    @property
    def n_vs(self) -> int:
        return int(self.valid.sum())

    @property
    def n_slopes(self) -> int:
        return 2 * self.n_gs * self.n_vs


def pupil_mask(n: int, D: float, obstruction: float, supersample: int = 64) -> np.ndarray:
    """Valid-subaperture rule: a subaperture is kept when at least half of its
    area lies inside the annular pupil (outer diameter D, inner obstruction*D).
    Area fractions are measured on a supersample x supersample point grid."""
    return _pupil_mask(int(n), float(D), float(obstruction), int(supersample)).copy()


@functools.lru_cache(maxsize=32)
def _pupil_mask(n: int, D: float, obstruction: float, supersample: int) -> np.ndarray:
    d = D / n
    t = (np.arange(supersample) + 0.5) / supersample
    valid = np.zeros((n, n), dtype=bool)
    for i in range(n):
        y = (i - n / 2 + t) * d
        for j in range(n):
            x = (j - n / 2 + t) * d
            X, Y = np.meshgrid(x, y)
            r = np.hypot(X, Y)
            inside = (r <= D / 2) & (r >= obstruction * D / 2)
            valid[i, j] = inside.mean() >= 0.5
    return valid


def ring(n_gs: int, radius_rad: float) -> np.ndarray:
    """Guide stars evenly spaced on a ring, the first at position angle 0 (+x)."""
    ang = 2.0 * np.pi * np.arange(n_gs) / n_gs
    return np.stack([radius_rad * np.cos(ang), radius_rad * np.sin(ang)], axis=1)


def lgs3_10x10(pad_L: int = 20) -> Workload:
    """8 m, 10x10, 3 LGS on a 30 arcsec ring, 2 layers (Table 1 geometry, reduced)."""
    n, D, obs = 10, 8.0, 0.30
    return Workload(
        name="lgs3_10x10", n=n, D=D, obstruction=obs, gs=ring(3, 30 * ARCSEC), h_lgs=90e3,
        h=np.array([0.0, 10e3]), w=np.array([0.7, 0.3]), r0=0.15, L0=25.0,
        noise_var=0.1, pad_L=pad_L, valid=pupil_mask(n, D, obs))


def lgs3_10x10_family(index: int, pad_L: int = 20) -> Workload:
    """Systems of the 10x10 / 3 LGS geometry with a random atmosphere, for
    training the learned preconditioner: the two layers of lgs3_10x10 with the
    ground-layer weight uniform in [0.5, 0.9] and r0 uniform in [0.10, 0.25] m
    (seed SEED + 500 + index).  Index -1 is lgs3_10x10 itself."""
    if index < 0:
        return lgs3_10x10(pad_L=pad_L)
    u = np.random.default_rng(SEED + 500 + int(index)).random(2)
    w0 = 0.5 + 0.4 * float(u[0])
    wl = lgs3_10x10(pad_L=pad_L)
    wl.name = f"lgs3_10x10_v{index}"
    wl.w = np.array([w0, 1.0 - w0])
    wl.r0 = 0.10 + 0.15 * float(u[1])
    return wl


def c2_profile(seed: int = SEED, n_layer: int = 35):
    """Synthetic 35-layer profile: geometric altitudes 30 m .. 26.5 km and
    weights proportional to exp(-h / 5 km) (0.75 + 0.5 u), u ~ U(0, 1), normalised."""
    k = np.arange(n_layer)
    h = 30.0 * (26500.0 / 30.0) ** (k / (n_layer - 1))
    u = np.random.default_rng(seed).random(n_layer)
    w = np.exp(-h / 5000.0) * (0.75 + 0.5 * u)
    return h, w / w.sum()


def lgs6_74x74(pad_L: int = 148) -> Workload:
    """39 m, 74x74, 6 LGS on a 60 arcsec ring, 35 layers (Table 2 geometry)."""
    n, D, obs = 74, 39.0, 0.28
    h, w = c2_profile()
    return Workload(
        name="lgs6_74x74", n=n, D=D, obstruction=obs, gs=ring(6, 60 * ARCSEC), h_lgs=90e3,
        h=h, w=w, r0=0.157, L0=25.0, noise_var=0.1, pad_L=pad_L,
        valid=pupil_mask(n, D, obs))


def lgs6_74x74_family(index: int, pad_L: int = 256) -> Workload:
    """Distinct systems of the 74x74 / 6 LGS geometry for batched products: the
    same pupil and asterism, the 35 altitudes of lgs6_74x74, layer weights drawn
    with seed SEED + 1 + index and r0 uniform in [0.10, 0.25] m from the same
    generator.  Index -1 is lgs6_74x74 itself (at this pad_L)."""
    if index < 0:
        return lgs6_74x74(pad_L=pad_L)
    n, D, obs = 74, 39.0, 0.28
    seed = SEED + 1 + int(index)
    h, w = c2_profile(seed=seed)
    r0 = 0.10 + 0.15 * float(np.random.default_rng(seed).random(36)[35])
    return Workload(
        name=f"lgs6_74x74_v{index}", n=n, D=D, obstruction=obs, gs=ring(6, 60 * ARCSEC), h_lgs=90e3,
        h=h, w=w, r0=r0, L0=25.0, noise_var=0.1, pad_L=pad_L,
        valid=pupil_mask(n, D, obs))


def uneven_family(index: int) -> Workload:
    """Uneven systems for batched solves: grid n from (40, 60, 74, 84) in turn,
    4-8 LGS at 90 km on a 40-70 arcsec ring, 10-35 layers (geometric altitudes
    30 m - 26.5 km, weights as c2_profile with seed SEED + 100 + index), r0 in
    [0.10, 0.25] m, noise variance in [0.01, 0.5] rad^2, 28 % obstruction on a
    pupil of 0.527 m per subaperture, L the smallest power of two >= 2n."""
    rng = np.random.default_rng(SEED + 100 + int(index))
    n = (40, 60, 74, 84)[int(index) % 4]
    n_gs = int(rng.integers(4, 9))
    n_layer = int(rng.integers(10, 36))
    h, w = c2_profile(seed=SEED + 100 + int(index), n_layer=n_layer)
    D = 0.52703 * n
    L = 1 << (2 * n - 1).bit_length()
    return Workload(
        name=f"uneven_{index}_n{n}_g{n_gs}_l{n_layer}", n=n, D=D, obstruction=0.28,
        gs=ring(n_gs, float(rng.uniform(40, 70)) * ARCSEC), h_lgs=90e3, h=h, w=w,
        r0=float(rng.uniform(0.10, 0.25)), L0=25.0, noise_var=float(rng.uniform(0.01, 0.5)), pad_L=L,
        valid=pupil_mask(n, D, 0.28))


def tiny(n: int = 4, n_gs: int = 2, lgs: bool = True, n_layer: int = 2,
         pad_L: Optional[int] = None, seed: int = 0, mask: str = "random",
         radius_arcsec: float = 40.0, D: Optional[float] = None) -> Workload:
    """Small seeded workload for exhaustive checks.  mask: 'full', 'random'
    (each subaperture kept with probability 0.7, at least one kept) or 'pupil'."""
    rng = np.random.default_rng(seed)
    D = float(D if D is not None else 0.5 * n)
    if mask == "full":
        valid = np.ones((n, n), bool)
    elif mask == "pupil":
        valid = pupil_mask(n, D, 0.2)
    else:
        valid = rng.random((n, n)) < 0.7
        if not valid.any():
            valid[rng.integers(n), rng.integers(n)] = True
    h = np.sort(rng.random(n_layer)) * 15e3
    h[0] = 0.0
    w = 0.5 + rng.random(n_layer)
    w /= w.sum()
    gs = ring(n_gs, radius_arcsec * ARCSEC)
    gs = gs + rng.normal(scale=3 * ARCSEC, size=gs.shape)
    return Workload(
        name=f"tiny_n{n}_g{n_gs}_{'lgs' if lgs else 'ngs'}_s{seed}", n=n, D=D,
        obstruction=0.0, gs=gs, h_lgs=(90e3 if lgs else math.inf), h=h, w=w,
        r0=0.12 + 0.1 * rng.random(), L0=20.0 + 10 * rng.random(),
        noise_var=0.05 + 0.2 * rng.random(), pad_L=int(pad_L if pad_L else 2 * n - 1),
        valid=valid)


# ----------------------------------------------------------------------------
# measured slopes
# ----------------------------------------------------------------------------

def gaussian_slopes(wl: Workload, seed: int = SEED, frames: int = 1) -> np.ndarray:
    """White Gaussian slope vectors (frames, n_slopes), unit variance."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((frames, wl.n_slopes))


_PSD_COEFF = 0.022895587108555  # (24/5 Gamma(6/5))^(5/6) Gamma(11/6)^2 / (2 pi^(11/3))


def _phase_screen(rng, N, dx, r0, L0):
    """Periodic von Karman phase screen, N x N samples of spacing dx [m], in rad."""
    fx = np.fft.fftfreq(N, dx)
    FX, FY = np.meshgrid(fx, fx)
    psd = _PSD_COEFF * r0 ** (-5.0 / 3.0) * (FX ** 2 + FY ** 2 + 1.0 / L0 ** 2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    df = 1.0 / (N * dx)
    c = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * np.sqrt(psd) * df
    return np.real(np.fft.ifft2(c)) * N * N


def _bilinear(screen, dx, x, y):
    N = screen.shape[0]
    fx = x / dx + N / 2
    fy = y / dx + N / 2
    j0 = np.floor(fx).astype(int)
    i0 = np.floor(fy).astype(int)
    tx = fx - j0
    ty = fy - i0
    j0 %= N
    i0 %= N
    j1 = (j0 + 1) % N
    i1 = (i0 + 1) % N
    return ((1 - tx) * (1 - ty) * screen[i0, j0] + tx * (1 - ty) * screen[i0, j1]
            + (1 - tx) * ty * screen[i1, j0] + tx * ty * screen[i1, j1])


def turbulent_slopes(wl: Workload, seed: int = SEED, frames: int = 1,
                     noise: bool = True) -> np.ndarray:
    """Slopes measured through seeded von Karman layers (frames, n_slopes).

    Each layer k is an FFT phase screen with r0_k^(-5/3) = w_k r0^(-5/3).  Along
    guide star j the layer is crossed at  c_k * x + h_k * alpha_j  with the cone
    factor c_k = 1 - h_k / h_lgs (1 for natural guide stars).  A slope is the
    phase difference between the two edge midpoints of a subaperture (x: right
    minus left edge, y: top minus bottom edge), plus N(0, noise_var) noise.
    Vector layout: sensor-major, x slopes then y slopes, valid subapertures in
    row-major order."""
    rng = np.random.default_rng(seed)
    n, d = wl.n, wl.d
    idx = np.flatnonzero(wl.valid.ravel())
    ii, jj = idx // n, idx % n
    cx = (jj - (n - 1) / 2.0) * d
    cy = (ii - (n - 1) / 2.0) * d
    reach = wl.D + 2 * float(np.max(wl.h)) * float(np.max(np.abs(wl.gs))) + 2 * d
    dx = d / 2.0
    N = 1 << int(math.ceil(math.log2(max(4 * reach, 4 * wl.L0) / dx)))
    out = np.zeros((frames, wl.n_slopes))
    for f in range(frames):
        s = np.zeros((wl.n_gs, 2, idx.size))
        for k in range(wl.n_layer):
            scr = _phase_screen(rng, N, dx, wl.r0 * wl.w[k] ** (-3.0 / 5.0), wl.L0)
            c = 1.0 if math.isinf(wl.h_lgs) else 1.0 - wl.h[k] / wl.h_lgs
            for g in range(wl.n_gs):
                ox, oy = wl.h[k] * wl.gs[g, 0], wl.h[k] * wl.gs[g, 1]
                px = c * cx + ox
                py = c * cy + oy
                e = c * d / 2.0
                s[g, 0] += _bilinear(scr, dx, px + e, py) - _bilinear(scr, dx, px - e, py)
                s[g, 1] += _bilinear(scr, dx, px, py + e) - _bilinear(scr, dx, px, py - e)
        v = s.reshape(-1)
        if noise:
            v = v + math.sqrt(wl.noise_var) * rng.standard_normal(v.size)
        out[f] = v
    return out


# ----------------------------------------------------------------------------
# elongated-spot noise
# ----------------------------------------------------------------------------
def elongated_noise(wl: Workload, elongation: float = 3.0, seed: int = SEED):
    """Slope noise of elongated LGS spots (§2.F): per valid subaperture a 2x2
    x-y noise covariance with principal axes along and across the radial
    direction from the pupil centre (laser launched on axis), variance
    sigma^2 (1 + e (rho / R)^2) along it and sigma^2 across it, e = elongation
    times a seeded per-sensor factor in [0.8, 1.2].  Returns (var, cov_xy):
    var (n_slopes,) in the slope-vector layout, cov_xy (n_gs, n_vs)."""
    rng = np.random.default_rng(seed)
    n, d = wl.n, wl.d
    idx = np.flatnonzero(wl.valid.ravel())
    ii, jj = idx // n, idx % n
    cx = (jj - (n - 1) / 2.0) * d
    cy = (ii - (n - 1) / 2.0) * d
    rho2 = (cx ** 2 + cy ** 2) / (wl.D / 2.0) ** 2
    th = np.arctan2(cy, cx)
    var = np.zeros((wl.n_gs, 2, idx.size))
    cov = np.zeros((wl.n_gs, idx.size))
    for g in range(wl.n_gs):
        e = elongation * (0.8 + 0.4 * rng.random())
        par = wl.noise_var * (1.0 + e * rho2)
        per = np.full(idx.size, wl.noise_var)
        c, s = np.cos(th), np.sin(th)
        var[g, 0] = par * c * c + per * s * s
        var[g, 1] = par * s * s + per * c * c
        cov[g] = (par - per) * s * c
    return var.reshape(-1), cov


def correlated_noise(var: np.ndarray, cov_xy: np.ndarray, seed: int = SEED) -> np.ndarray:
    """One seeded sample of slope noise with the given per-slope variances and
    x-y covariances (same layouts as elongated_noise)."""
    rng = np.random.default_rng(seed)
    G, nv = cov_xy.shape
    v = var.reshape(G, 2, nv)
    # 2x2 Cholesky per subaperture
    l11 = np.sqrt(v[:, 0])
    l21 = cov_xy / l11
    l22 = np.sqrt(v[:, 1] - l21 ** 2)
    z = rng.standard_normal((2, G, nv))
    out = np.zeros((G, 2, nv))
    out[:, 0] = l11 * z[0]
    out[:, 1] = l21 * z[0] + l22 * z[1]
    return out.reshape(-1)
