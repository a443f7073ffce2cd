"""FP64 CPU oracle for the Toeplitz spatio-angular MMSE tomographic reconstructor
(Ono et al., "Fast Iterative Tomographic Wave-front Estimation with Recursive
Toeplitz Reconstructor Structure for Large Scale Systems", JOSA A 2018).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything under this package;
only the test suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code with the HIP path: the only module both sides read
is the seeded input generator ``workloads``, which holds no arithmetic of the
method.

Every function is written for clarity, in float64, and cites the passage of
the paper it follows.  Modules:

  vonkarman   phase structure function D(r) and PSD constant (App. A.1, A.2)
  geometry    subaperture / phase-point coordinates, LGS cone scaling (§2, §2.D)
  covariance  Hudgin-like slope-slope and phase-slope covariances, dense
              Sigma_ss, Sigma_phi_s and the system matrix (App. A.2, §2.D, §2.F)
  toeplitz    the 2RBT matrix-vector product by circulant embedding, step by
              step (§2.E: shuffle, FFT, element-wise product, inverse FFT,
              reshuffle; fused over blocks as in the Sigma_ss zeta equation)
  solve       Cholesky solve of (Sigma_ss + Sigma_eta) zeta = s, plain CG and
              preconditioned CG (§2.C, §2.G)
  precond     block-circulant preconditioner: the positive part of the
              per-frequency embedded spectra plus sigma^2, inverted (§2.E
              embedding; preconditioning is left open in §2.G)
  projection  the LGS phase-slope product through per-layer grids with
              bilinear interpolation (§2.D "Phase-Slope Covariance Matrix",
              §2.E LGS equation), plus the exact dense form for comparison
  opcount     operation-count and compression formulas (§2.D, §2.E)
  learned     learned preconditioner P = K^T K, K a masked four-layer linear
              CNN over the slope maps (triangular, so log|det K| is exact),
              its Kaporin-number training objective on (residual, exact
              solution) pairs, gradient and Adam step (§2.G leaves
              preconditioning open); flexible PCG is solve.fpcg

Parity status: every function is pinned by a CPU test (tests/test_oracle_*.py)
against closed forms, library special functions, brute force or invariants;
none is "parity unpinned".
"""
