"""The 2RBT matrix-vector product by circulant embedding (§2.E), in float64.

Steps, in the order §2.E gives them, for a block Theta (2RBT, unique elements t)
and a vector x on the n x n subaperture grid:

  1. shuffle  b = S1 x        x placed on the top-left n x n corner of an L x L
                              array (zeros elsewhere);
  2. FFT      b~ = F[b]
  3. product  c~ = t~ . b~    t~ is the FFT of the embedded unique elements;
  4. inverse  c  = F^-1[c~]
  5. reshuffle y = S2 c       the top-left n x n corner, back to vector order.

Reading of the garbled shuffle rules (the printed index ranges read
"0 >= i, j >= n" and the ordering of t is only given in a figure): the
equivalent two-dimensional circulant embedding is used with any side
L >= 2n - 1.  The unique elements are stored reflected,
K[(-u) mod L, (-v) mod L] = t(u, v), so that the circular convolution of K with
b reproduces sum_b Theta[a, b] x_b without wrap-around.  The paper's own
one-dimensional form (length (2n-1)^2, reversed shuffle) is the special case
L = 2n - 1 read out in a different order; a test checks both against the dense
product.

For Sigma_ss zeta (§2.E, slope-slope equation) the forward transforms of the
C = 2 N_gs channels are computed once, the element-wise products are summed over
the input channel before one inverse transform per output channel, and W_s
restricts to valid subapertures (§2.F).
"""
import numpy as np

from . import geometry as G


def embed_kernel(t, L):
    """(2n-1, 2n-1) unique elements t[v+n-1, u+n-1] -> L x L reflected embedding."""
    m = t.shape[0]
    n = (m + 1) // 2
    if L < 2 * n - 1:
        raise ValueError("L must be >= 2n-1")
    K = np.zeros((L, L))
    lag = np.arange(-(n - 1), n)
    rows = (-lag) % L
    K[np.ix_(rows, rows)] = t
    return K


def kernel_spectra(tables, n_gs, L):
    """t~_{ab} = rfft2 of the embedded unique elements, for every ordered channel
    pair (a, b), a = 2*gi + p, b = 2*gj + q.  Returns (C, C, L, L//2+1) complex."""
    C = 2 * n_gs
    out = None
    for (gi, gj, p, q), t in tables.items():
        spec = np.fft.rfft2(embed_kernel(t, L))
        if out is None:
            out = np.zeros((C, C) + spec.shape, dtype=np.complex128)
        out[2 * gi + p, 2 * gj + q] = spec
    return out


def shuffle(xv, valid, L):
    """Step 1 (with W_s^T): valid-slope vector of one channel -> L x L array."""
    n = valid.shape[0]
    b = np.zeros((L, L))
    full = np.zeros(n * n)
    full[G.valid_index(valid)] = xv
    b[:n, :n] = full.reshape(n, n)
    return b


def reshuffle(c, valid):
    """Step 5 (with W_s): top-left n x n corner -> valid-slope vector."""
    n = valid.shape[0]
    return c[:n, :n].ravel()[G.valid_index(valid)]


def slope_matvec(spectra, valid, zeta, L):
    """W_s Sigma_ss W_s^T zeta by the fused 2RBT product of §2.E."""
    C = spectra.shape[0]
    nv = int(valid.sum())
    z = np.asarray(zeta, dtype=np.float64).reshape(C, nv)
    zt = [np.fft.rfft2(shuffle(z[b], valid, L)) for b in range(C)]     # steps 1-2
    y = np.zeros((C, nv))
    for a in range(C):
        acc = np.zeros_like(zt[0])
        for b in range(C):
            acc += spectra[a, b] * zt[b]                                 # step 3, summed
        c = np.fft.irfft2(acc, s=(L, L))                                 # step 4
        y[a] = reshuffle(c, valid)                                       # step 5
    return y.reshape(-1)


class ToeplitzOperator:
    """A = W_s (Sigma_ss + sigma^2 I) W_s^T applied through slope_matvec."""

    def __init__(self, wl, tables=None, L=None, noise_var=None):
        from .covariance import kernel_tables
        self.L = int(L if L is not None else wl.pad_L)
        self.valid = wl.valid
        self.noise_var = wl.noise_var if noise_var is None else noise_var
        self.tables = kernel_tables(wl) if tables is None else tables
        self.spectra = kernel_spectra(self.tables, wl.n_gs, self.L)
        self.n = wl.n_slopes

    def __call__(self, x):
        return slope_matvec(self.spectra, self.valid, x, self.L) + self.noise_var * np.asarray(x)
