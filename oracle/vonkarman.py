"""von Karman phase statistics (App. A.1 phase PSD, App. A.2 structure function).

Readings of the printed formulas (the printed text is garbled in two places):

* The structure function prints the factor (r0/L0)^(5/6) in front of the Bessel
  term; the bracket only vanishes at r = 0 (as any structure function must) when
  that factor is (r/L0)^(5/6).  With x = 2 pi r / L0 this is the same as
  (2^(1/6) / Gamma(5/6)) x^(5/6) K_{5/6}(x).
* The printed leading constant 0.17253 differs from the closed form
  Gamma(11/6) Gamma(5/6) pi^(-8/3) (24/5 Gamma(6/5))^(5/6) = 0.1726287 in the
  fourth digit; the closed form is used (it is what makes D(r) match the
  Kolmogorov law 6.88 (r/r0)^(5/3) at small r and 2 x phase variance at large r).
* The printed PSD constant 0.029 is inconsistent with the structure function by
  a factor 1.27; the consistent value (24/5 Gamma(6/5))^(5/6) Gamma(11/6)^2 /
  (2 pi^(11/3)) = 0.022896 is used.  The PSD is only used to generate test
  phase screens.

Units: r0 is given at the wavelength at which phase is expressed (500 nm);
D is in rad^2.
"""
import numpy as np
from scipy.special import gamma, kv

NU = 5.0 / 6.0

#: closed-form coefficient of (L0/r0)^(5/3) in D(r)   (App. A.2, structure function)
C_D = gamma(11.0 / 6.0) * gamma(5.0 / 6.0) / np.pi ** (8.0 / 3.0) * (24.0 / 5.0 * gamma(6.0 / 5.0)) ** (5.0 / 6.0)

#: Kolmogorov small-separation coefficient: D(r) -> C_KOLMO (r/r0)^(5/3)
C_KOLMO = 2.0 * (24.0 / 5.0 * gamma(6.0 / 5.0)) ** (5.0 / 6.0)

#: PSD coefficient of r0^(-5/3) (f^2 + L0^-2)^(-11/6)   (App. A.1, von Karman PSD)
C_PSD = (24.0 / 5.0 * gamma(6.0 / 5.0)) ** (5.0 / 6.0) * gamma(11.0 / 6.0) ** 2 / (2.0 * np.pi ** (11.0 / 3.0))


def structure_function(r, r0, L0):
    """D(r) for von Karman turbulence, App. A.2 (reading: (r/L0)^(5/6), exact constant).

    r may be an array of separations in metres (>= 0).  D(0) = 0.
    """
    r = np.asarray(r, dtype=np.float64)
    x = 2.0 * np.pi * r / L0
    out = np.zeros_like(x)
    nz = x > 0
    xb = x[nz]
    bracket = 1.0 - (2.0 ** (1.0 - NU) / gamma(NU)) * xb ** NU * kv(NU, xb)
    out[nz] = C_D * (L0 / r0) ** (5.0 / 3.0) * bracket
    return out


def phase_variance(r0, L0):
    """sigma_phi^2 = D(infinity) / 2 (App. A.2: the bracket tends to 1)."""
    return 0.5 * C_D * (L0 / r0) ** (5.0 / 3.0)


def phase_psd(f, r0, L0):
    """von Karman phase PSD Phi(f), App. A.1 (reading: constant 0.022896)."""
    f = np.asarray(f, dtype=np.float64)
    return C_PSD * r0 ** (-5.0 / 3.0) * (f * f + 1.0 / (L0 * L0)) ** (-11.0 / 6.0)
