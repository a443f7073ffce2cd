"""Block-circulant preconditioner of the masked 2RBT system, in float64.

The paper leaves preconditioning of its Toeplitz system open (§2.G, and the
conclusion names it as the remaining challenge).  This is the classical
choice for a block-Toeplitz operator that is applied through circulant
embedding (§2.E): invert the embedding itself, frequency by frequency.

With the same embedding as the product (side L, reflected unique elements,
`oracle.toeplitz.kernel_spectra`) the C x C per-frequency matrix M(f) of the
2C = 2 N_gs channel spectra is Hermitian, and the embedded block-circulant
operator is F^-1 diag_f(M(f)) F.  A circulant embedding of a covariance need
not be positive semi-definite, so M(f) is replaced by its positive part
M_+(f) (negative eigenvalues set to zero) before the noise variance is added:

    P r = W_s S2 F^-1 [ (M_+(f) + sigma^2 I)^-1 F[S1 W_s^T r] ]

i.e. the restriction of the inverse of the positive, noise-regularised
embedding to the valid subapertures, applied by the same shuffle / transform
/ per-frequency product / inverse / reshuffle steps as the product itself.
P is symmetric positive definite (a restriction of an SPD operator), so plain
preconditioned CG applies.  sigma^2 is the scalar noise variance (the mean of
per-slope variances when those are given).

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
import numpy as np

from .toeplitz import kernel_spectra, slope_matvec


def inverse_spectra(spectra, noise_var):
    """(C, C, L, Lh) spectra -> per-frequency (M_+ + sigma^2 I)^-1, same shape."""
    Mf = np.moveaxis(spectra, (0, 1), (-2, -1))              # (L, Lh, C, C)
    Mf = 0.5 * (Mf + np.conj(np.swapaxes(Mf, -1, -2)))       # Hermitian part (rounding only)
    lam, V = np.linalg.eigh(Mf)
    lam = np.maximum(lam, 0.0) + noise_var
    inv = (V / lam[..., None, :]) @ np.conj(np.swapaxes(V, -1, -2))
    return np.moveaxis(inv, (-2, -1), (0, 1))


class CirculantPreconditioner:
    """z = P r for the workload's system at FFT side L (default: its pad_L)."""

    def __init__(self, wl, tables=None, L=None, noise_var=None):
        from .covariance import kernel_tables
        self.L = int(L if L is not None else wl.pad_L)
        self.valid = wl.valid
        tables = kernel_tables(wl) if tables is None else tables
        nv = wl.noise_var if noise_var is None else noise_var
        self.noise_var = float(np.mean(nv))
        self.spectra = kernel_spectra(tables, wl.n_gs, self.L)
        self.inv = inverse_spectra(self.spectra, self.noise_var)

    def __call__(self, r):
        return slope_matvec(self.inv, self.valid, r, self.L)
