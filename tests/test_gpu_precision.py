"""Precision forms of the persistent solver through the C ABI: the column DFT
stages of the 2RBT product on the matrix cores with FP16 (TT_PREC_F16) or
BF16 (TT_PREC_BF16) operands and FP32 accumulation, FP32 vectors and
per-frequency products, FP64 residual refinement.

Bounds.  The first iterates of a low-precision form differ from the FP32 ones
by the operand rounding of the column transforms (twiddles and block-scaled
data, unit roundoff u = 2^-11 for FP16, 2^-8 for BF16); an iterate carries a
few such roundings, so the bound is 4u: 1.95e-3 (FP16), 1.56e-2 (BF16).
Full solves must report an honest status: TT_OK only when the FP64 true
residual, recomputed here with the oracle's dense matrix, is at or under tol;
otherwise TT_NOT_CONVERGED, with rel_residual equal (to the norm-wise FP64
rounding bound of s - A z, 1e-11 (||A|| ||z|| + ||s||) / ||s||, the accuracy
the FP64 product is held to elsewhere) to the residual of the returned
iterate."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, say, torch_dev

pytestmark = pytest.mark.gpu

FORMS = {2: 2.0 ** -11, 3: 2.0 ** -8}   # precision -> unit roundoff


@pytest.fixture(scope="module")
def c1sys():
    wl = W.lgs3_10x10()
    ctx, k = make_system(wl, target=True)
    return wl, ctx, k


@pytest.mark.parametrize("precision", sorted(FORMS))
def test_first_iterates_within_operand_rounding(c1sys, precision):
    import torch
    from paper_1806_07938_amd.tt import TT_NOT_CONVERGED
    wl, ctx, k = c1sys
    s = torch.tensor(W.turbulent_slopes(wl)[0].astype(np.float32), device=torch_dev())
    for it in (1, 2, 3):
        z32, _, _ = ctx.solve(s, tol=1e-12, max_iter=it, precision=0, allow=(0, TT_NOT_CONVERGED))
        zlo, _, info = ctx.solve(s, tol=1e-12, max_iter=it, precision=precision, allow=(0, TT_NOT_CONVERGED))
        a, b = z32.cpu().numpy(), zlo.cpu().numpy()
        d = np.linalg.norm(b - a) / np.linalg.norm(a)
        say("precision", precision, "iterations", it, "difference to FP32", d)
        assert info.iterations == it
        assert d < 4 * FORMS[precision]


@pytest.mark.parametrize("precision", sorted(FORMS))
def test_full_solve_status_is_honest(c1sys, precision):
    import torch
    from oracle.covariance import system_matrix
    from paper_1806_07938_amd.tt import TT_NOT_CONVERGED
    wl, ctx, k = c1sys
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    z, _, info = ctx.solve(torch.tensor(s, device=torch_dev()), tol=1e-6, precision=precision,
                           allow=(0, TT_NOT_CONVERGED))
    zz = z.cpu().numpy()
    assert np.all(np.isfinite(zz))
    A = system_matrix(wl)
    res = np.linalg.norm(s - A @ zz) / np.linalg.norm(s)
    say("precision", precision, "status", info.status, "iterations", info.iterations, "refinements",
        info.refinements, "library residual", info.rel_residual, "oracle residual", res)
    # both residuals are FP64 evaluations of s - A z: they agree to the
    # norm-wise rounding bound of that product, relative to ||A|| ||z|| + ||s||
    scale = (np.linalg.norm(A, 2) * np.linalg.norm(zz) + np.linalg.norm(s)) / np.linalg.norm(s)
    assert abs(info.rel_residual - res) <= 1e-11 * scale
    if info.status == 0:
        assert res <= 1.01e-6
    else:
        assert info.status == TT_NOT_CONVERGED and info.rel_residual > 1e-6


@pytest.mark.parametrize("precision", sorted(FORMS))
def test_batched_pcg_with_half_preconditioner_spectra_converges(c1sys, precision):
    """TT_SOLVER_BATCHED + TT_PRECOND_CIRCULANT with FP16 / BF16: only the
    preconditioner's spectra are stored in reduced precision; the FP32 product
    and the FP64 residual replacement keep the method exact, so the solve
    reaches 1e-6 (and 1e-10, config 1's tolerance) like the FP32 form."""
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT, SOLVER_BATCHED
    wl, ctx, k = c1sys
    A = system_matrix(wl)
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    st = torch.tensor(s, device=torch_dev())
    zref = cholesky_solve(A, s.astype(np.float64))
    for tol in (1e-6, 1e-10):
        z, phi, info = ctx.solve(st, tol=tol, precision=precision, solver=SOLVER_BATCHED,
                                 preconditioner=PRECOND_CIRCULANT)
        _, _, info32 = ctx.solve(st, tol=tol, solver=SOLVER_BATCHED, preconditioner=PRECOND_CIRCULANT)
        zz = z.cpu().numpy()
        res = np.linalg.norm(s - A @ zz) / np.linalg.norm(s)
        err = np.linalg.norm(zz - zref) / np.linalg.norm(zref)
        say(f"precision {precision} tol {tol:g}: {info.iterations} iterations (FP32 spectra {info32.iterations}), "
            f"oracle residual {res:.2e}, zeta error {err:.2e}")
        assert info.status == 0 and res <= 1.01 * tol
        if tol == 1e-10:
            assert err < 1e-5


def test_low_precision_needs_persistent_solver(c1sys):
    import torch
    from paper_1806_07938_amd import TTError
    from paper_1806_07938_amd.tt import TT_INVALID_ARG
    wl, ctx, k = c1sys
    s = torch.zeros(wl.n_slopes, dtype=torch.float32, device=torch_dev())
    for precision in sorted(FORMS):
        with pytest.raises(TTError) as e:
            ctx.solve(s, precision=precision, solver=1)
        assert e.value.status == TT_INVALID_ARG
    with pytest.raises(TTError) as e:
        ctx.solve(s, precision=7)
    assert e.value.status == TT_INVALID_ARG
