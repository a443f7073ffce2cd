"""Pins of the structure function D(r) (App. A.2) and PSD constant (App. A.1)
against closed forms and an independent route (the PSD Hankel integral)."""
import json
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import j0

from oracle import vonkarman as VK

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


def test_D_zero_and_monotone():
    r = np.linspace(0, 200, 2001)
    D = VK.structure_function(r, 0.15, 25.0)
    assert D[0] == 0.0
    assert np.all(np.diff(D) >= -1e-12 * D.max())
    assert np.all(np.diff(D[r < 60]) > 0)


def test_constant_matches_printed_to_3_digits():
    printed = GOLD["structure_function_constant_printed"]["value"]
    assert abs(VK.C_D - printed) / printed < 1e-3
    assert abs(VK.C_D - 0.1726286598) < 1e-9


@pytest.mark.parametrize("r0,L0", [(0.15, 25.0), (0.1, 10.0), (0.25, 50.0)])
def test_kolmogorov_limit(r0, L0):
    # D(r) / (6.88 (r/r0)^(5/3)) -> 1 as x = 2 pi r / L0 -> 0, and the deficit
    # shrinks as x^(1/3) (the next term of the small-x expansion is O(x^2)
    # against the leading x^(5/3)).  Absolute precision of D is ~1e-13 rad^2, so
    # x is kept >= 1e-6, where the relative rounding error is still < 1e-4.
    def deficit(x):
        r = x * L0 / (2 * np.pi)
        return 1 - VK.structure_function(np.array([r]), r0, L0)[0] / (6.883877182293812 * (r / r0) ** (5 / 3))
    d5, d7 = deficit(1e-4), deficit(1e-6)
    assert 0 < d7 < d5 < 0.05
    assert abs(d7 / d5 - (1e-2) ** (1 / 3)) < 0.01


def test_saturation_is_twice_phase_variance():
    r0, L0 = 0.15, 25.0
    D = VK.structure_function(np.array([50 * L0]), r0, L0)[0]
    assert abs(D - 2 * VK.phase_variance(r0, L0)) / D < 1e-12
    # 0.0863 (L0/r0)^(5/3): textbook von Karman phase variance coefficient
    assert abs(VK.phase_variance(1.0, 1.0) - 0.0863143) < 1e-6


@pytest.mark.parametrize("r", [0.05, 0.1, 0.8, 5.0, 30.0])
def test_matches_psd_hankel_integral(r):
    # D(r) = 2 int_0^inf (1 - J0(2 pi f r)) Phi(f) 2 pi f df: an independent route
    # from the PSD of App. A.1 (reading: constant 0.022896) to D.
    r0, L0 = 0.15, 25.0

    def integrand(f):
        return 2 * (1 - j0(2 * np.pi * f * r)) * VK.phase_psd(f, r0, L0) * 2 * np.pi * f

    brk = [0, 1 / L0, 10 / L0, 1 / r, 10 / r, 100 / r]
    brk = sorted(set(brk))
    total = 0.0
    for a, b in zip(brk[:-1], brk[1:]):
        total += integrate.quad(integrand, a, b, limit=400, epsabs=0, epsrel=1e-12)[0]
    total += integrate.quad(integrand, brk[-1], np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
    D = VK.structure_function(np.array([r]), r0, L0)[0]
    assert abs(total - D) / D < 1e-8


def test_printed_psd_constant_is_inconsistent():
    # The printed 0.029 gives D 27 % too large; the consistent constant is 0.022896.
    assert abs(VK.C_PSD - 0.0228955871) < 1e-9
    assert 1.2 < 0.029 / VK.C_PSD < 1.3
