"""Low-order mode removal (§2.F) through the C ABI against the oracle
(oracle.modes): the product M_s A M_s, the solve of the mode-removed system
(one launch per phase), and the projection M_phi W_phi Sigma_phi_s M_s zeta.

Tolerances as elsewhere: FP64 products to 1e-11 of the largest entry, FP32
to 3e-6; solves certified by the FP64 residual of the mode-removed system
(recomputed with the oracle's dense matrices) and within 1e-5 of the oracle's
solution; projections to 1e-5."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu

CASES = [dict(n=6, n_gs=2, lgs=True, n_layer=3, seed=4, pad_L=12),
         dict(n=7, n_gs=3, lgs=True, n_layer=2, seed=5, pad_L=16)]


def _wl(case):
    return W.tiny(**case) if isinstance(case, dict) else case()


@pytest.mark.parametrize("case", CASES + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_mode_removed_product(case):
    import torch
    from oracle.covariance import system_matrix
    from oracle.modes import slope_projector
    wl = _wl(case)
    ctx, k = make_system(wl, target=True)
    ctx.set_mode_removal(True)
    M = slope_projector(wl)
    A = system_matrix(wl)
    dev = torch_dev()
    x = np.random.default_rng(3).standard_normal(wl.n_slopes)
    assert rel_maxabs(ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy(), M @ A @ M @ x) < 1e-11
    x32 = x.astype(np.float32)
    y32 = ctx.matvec(torch.tensor(x32, device=dev)).cpu().numpy()
    assert rel_maxabs(y32, M @ A @ M @ x32.astype(np.float64)) < 3e-6
    ctx.set_mode_removal(False)
    assert rel_maxabs(ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy(), A @ x) < 1e-11


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("case", CASES + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_mode_removed_solve_and_projection(case, precision):
    import torch
    from oracle.covariance import system_matrix
    from oracle.modes import phase_projector, slope_projector, solve_mode_removed
    from oracle.projection import phi_paper_dense
    wl = _wl(case)
    ctx, k = make_system(wl, target=True)
    ctx.set_mode_removal(True)
    M = slope_projector(wl)
    A = system_matrix(wl)
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    s64 = s.astype(np.float64)
    tol = 1e-9
    z, phi, info = ctx.solve(torch.tensor(s, device=torch_dev()), tol=tol, precision=precision, solver=1)
    zz = z.cpu().numpy()
    Ms = M @ s64
    res = np.linalg.norm(Ms - M @ A @ M @ zz) / np.linalg.norm(Ms)
    zref = solve_mode_removed(A, M, s64)
    say("modes", wl.name, "precision", precision, "iterations", info.iterations, "residual", res)
    assert info.status == 0
    assert res <= 1.01 * tol
    assert abs(info.rel_residual - res) <= 1e-3 * tol
    assert np.linalg.norm(M @ zz - zz) <= 1e-12 * np.linalg.norm(zz)
    assert np.linalg.norm(zz - zref) <= 1e-5 * np.linalg.norm(zref)
    ref = phase_projector(wl) @ phi_paper_dense(wl, M @ zz.astype(np.float32).astype(np.float64))
    assert rel_maxabs(phi.cpu().numpy(), ref) < 1e-5


def test_mode_removal_errors():
    import torch
    from paper_1806_07938_amd import Context, TTError
    from paper_1806_07938_amd.tt import TT_INVALID_ARG, TT_NOT_READY
    wl = W.lgs3_10x10()
    with pytest.raises(TTError) as e:
        Context(0).set_mode_removal(True)
    assert e.value.status == TT_NOT_READY
    ctx, k = make_system(wl, target=False)
    ctx.set_mode_removal(True)
    s = torch.ones(wl.n_slopes, dtype=torch.float32, device=torch_dev())
    with pytest.raises(TTError) as e:
        ctx.solve(s, solver=0)
    assert e.value.status == TT_INVALID_ARG
