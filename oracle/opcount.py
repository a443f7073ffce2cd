"""Operation counts and compression factors of §2.D and §2.E (log base 2, FFT
cost a N log N; §4 uses a = 5).  Used for accounting only."""
import math


def compression_ss(n):
    """Unique / total elements of Sigma_ss: (2n-1)^2 n^-4 (§2.D)."""
    return (2 * n - 1) ** 2 / n ** 4


def compression_ps_ngs(n):
    """Sigma_phi_s, NGS: 4 (n+1)^-2 (§2.D)."""
    return 4.0 / (n + 1) ** 2


def compression_ps_lgs(n, n_gs, n_primes):
    """Sigma_phi_s, LGS: [sum_k (n'_k+n-1)^2] (n+1)^-2 n^-2 + 2 N_layer N_gs^-1 (n+1)^-2 (§2.D)."""
    nl = len(n_primes)
    return (sum((m + n - 1) ** 2 for m in n_primes) / ((n + 1) ** 2 * n ** 2)
            + 2.0 * nl / (n_gs * (n + 1) ** 2))


def ops_2rbt(m, n, a=5.0):
    """One m^2 x n^2 2RBT product: (m+n-1)^2 [4 a log(m+n-1) + 1] + m^2 + n^2 (§2.E)."""
    N = m + n - 1
    return N * N * (4 * a * math.log2(N) + 1) + m * m + n * n


def ops_ss(n, n_gs, a=5.0):
    """Sigma_ss zeta: 4 N_gs {(2n-1)^2 [2 a log(2n-1) + N_gs] + n^2} (§2.E)."""
    N = 2 * n - 1
    return 4 * n_gs * (N * N * (2 * a * math.log2(N) + n_gs) + n * n)


def reduction_ss(n, n_gs, a=5.0):
    """ops_ss / dense 4 N_gs^2 n^4 (§2.E)."""
    return ops_ss(n, n_gs, a) / (4.0 * n_gs ** 2 * n ** 4)


def ops_ps_ngs(n, n_gs, a=5.0):
    """NGS Sigma_phi_s zeta: 2N_gs[4n^2(2a log 2n + 1) + n^2] + 8 n^2 log 2n + (n+1)^2 (§2.E)."""
    L2 = math.log2(2 * n)
    return 2 * n_gs * (4 * n * n * (2 * a * L2 + 1) + n * n) + 8 * n * n * L2 + (n + 1) ** 2


def reduction_ps_ngs(n, n_gs, a=5.0):
    return ops_ps_ngs(n, n_gs, a) / (2.0 * n_gs * (n + 1) ** 2 * n ** 2)


def ops_ps_lgs(n, n_gs, n_layer, n_prime, a=5.0):
    """LGS Sigma_phi_s zeta, common n':
    2(n'+n-1)^2[(2N_gs+N_layer) a log(n'+n-1) + N_gs N_layer] + 2 N_gs n^2 + 4 N_layer (n+1)^2 (§2.E)."""
    N = n_prime + n - 1
    return (2 * N * N * ((2 * n_gs + n_layer) * a * math.log2(N) + n_gs * n_layer)
            + 2 * n_gs * n * n + 4 * n_layer * (n + 1) ** 2)


def reduction_ps_lgs(n, n_gs, n_layer, n_prime, a=5.0):
    return ops_ps_lgs(n, n_gs, n_layer, n_prime, a) / (2.0 * n_gs * (n + 1) ** 2 * n ** 2)
