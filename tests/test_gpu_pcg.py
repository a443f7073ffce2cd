"""GPU parity of the preconditioned persistent solver (TT_PRECOND_CIRCULANT)
against the oracle's block-circulant preconditioner and PCG, through the C ABI.

* First iterate: from x0 = 0, one iteration gives x1 = alpha0 P s with
  alpha0 = s.Ps / (Ps).A(Ps); the oracle computes P s with its own
  preconditioner (dense eigen-decomposition per frequency, FFTs), so this pins
  the library's preconditioner spectra (host Jacobi), their general Hermitian
  packing and the preconditioner column phase: to 1e-10 in FP64, 1e-5 in FP32.
* Full solves reach the oracle's Cholesky solution (FP64 true residual at or
  under tol, checked with the oracle's dense matrix; solution to 1e-5), in
  as many iterations as the oracle's PCG (FP64: within 5 %; FP32: restarts at
  the FP64 residual replacements allowed for), and at the 10x10 workload in
  fewer than plain CG.
* Shapes: tiny systems with ragged masks and odd paddings, the 10x10 / 3 LGS
  workload; the 74x74 workload is in test_gpu_74x74.py."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, say, torch_dev

pytestmark = pytest.mark.gpu

CASES = [dict(n=5, n_gs=2, lgs=True, n_layer=3, seed=4, pad_L=12),
         dict(n=7, n_gs=4, lgs=True, n_layer=2, seed=5, pad_L=16),
         dict(n=6, n_gs=1, lgs=False, n_layer=2, seed=6, pad_L=11)]


def _wl(case):
    return W.tiny(**case) if isinstance(case, dict) else case()


@pytest.mark.parametrize("precision,tol", [(1, 1e-10), (0, 1e-5)])
@pytest.mark.parametrize("case", CASES + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_first_iterate_is_alpha_P_s(case, precision, tol):
    import torch
    from oracle.covariance import system_matrix
    from oracle.precond import CirculantPreconditioner
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT, TT_NOT_CONVERGED
    wl = _wl(case)
    say("pcg first iterate", wl.name, "precision", precision)
    ctx, k = make_system(wl, target=False)
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    z, _, info = ctx.solve(torch.tensor(s, device=torch_dev()), tol=1e-14, max_iter=1, precision=precision,
                           preconditioner=PRECOND_CIRCULANT, allow=(0, TT_NOT_CONVERGED))
    assert info.iterations == 1
    A = system_matrix(wl)
    s64 = s.astype(np.float64)
    u = CirculantPreconditioner(wl)(s64)
    x1 = (s64 @ u) / (u @ (A @ u)) * u
    d = np.linalg.norm(z.cpu().numpy() - x1) / np.linalg.norm(x1)
    say("  difference", d)
    assert d < tol


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("case", CASES + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_pcg_solve_matches_cholesky(case, precision):
    import torch
    from oracle.covariance import system_matrix
    from oracle.precond import CirculantPreconditioner
    from oracle.solve import cg, cholesky_solve, pcg
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT
    wl = _wl(case)
    ctx, k = make_system(wl, target=True)
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    s64 = s.astype(np.float64)
    A = system_matrix(wl)
    tol = 1e-10 if precision == 1 else 1e-8
    z, phi, info = ctx.solve(torch.tensor(s, device=torch_dev()), tol=tol, precision=precision,
                             preconditioner=PRECOND_CIRCULANT)
    zz = z.cpu().numpy()
    res = np.linalg.norm(s64 - A @ zz) / np.linalg.norm(s64)
    zref = cholesky_solve(A, s64)
    _, k_pcg = pcg(lambda v: A @ v, CirculantPreconditioner(wl), s64, tol=tol)
    _, k_cg = cg(lambda v: A @ v, s64, tol=tol)
    say("pcg", wl.name, "precision", precision, "iterations", info.iterations, "oracle PCG", k_pcg, "oracle CG", k_cg,
        "refinements", info.refinements, "residual", res)
    assert info.status == 0
    assert res <= 1.01 * tol
    assert abs(info.rel_residual - res) <= 1e-3 * tol
    assert np.linalg.norm(zz - zref) <= 1e-5 * np.linalg.norm(zref)
    if precision == 1:   # FP64, no replacements: the iterates of the oracle's PCG up to rounding
        assert abs(info.iterations - k_pcg) <= max(2, 0.05 * k_pcg)
    else:                # FP32: each FP64 residual replacement restarts the recurrences
        assert info.iterations <= 1.5 * k_pcg + 10 * info.refinements
    if wl.name == "lgs3_10x10":  # the preconditioner pays at the 10x10 workload (311 -> 163 at 1e-6)
        assert info.iterations < 0.8 * k_cg


def test_pcg_zero_slopes_and_warm_start():
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT
    wl = W.lgs3_10x10()
    ctx, k = make_system(wl, target=False)
    dev = torch_dev()
    z, _, info = ctx.solve(torch.zeros(wl.n_slopes, dtype=torch.float32, device=dev), preconditioner=PRECOND_CIRCULANT)
    assert info.iterations == 0 and not np.any(z.cpu().numpy())
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    zref = cholesky_solve(system_matrix(wl), s.astype(np.float64))
    z, _, info = ctx.solve(torch.tensor(s, device=dev), x0=torch.tensor(zref, device=dev), tol=1e-6,
                           preconditioner=PRECOND_CIRCULANT)
    assert info.status == 0 and info.iterations == 0


def test_pcg_argument_errors():
    import torch
    from paper_1806_07938_amd import TTError
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT, TT_INVALID_ARG
    wl = W.lgs3_10x10()
    ctx, k = make_system(wl, target=False)
    s = torch.zeros(wl.n_slopes, dtype=torch.float32, device=torch_dev())
    for kw in (dict(solver=1), dict(precision=2), dict(precision=3)):
        with pytest.raises(TTError) as e:
            ctx.solve(s, preconditioner=PRECOND_CIRCULANT, **kw)
        assert e.value.status == TT_INVALID_ARG
    with pytest.raises(TTError) as e:
        ctx.solve(s, preconditioner=5)
    assert e.value.status == TT_INVALID_ARG
