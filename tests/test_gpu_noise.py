"""2x2 noise blocks of elongated LGS spots (§2.F) through the C ABI: the
products and every solver against the oracle's dense system with the same
Sigma_eta (oracle.covariance.noise_covariance: per-slope variances plus the
x-y covariance of each subaperture), and the argument / state errors.

Tolerances as the diagonal-noise tests: FP64 products to 1e-11 of the largest
entry, FP32 products to 3e-6, solves certified by the FP64 residual (checked
with the oracle's matrix) and within 1e-5 of the Cholesky solution."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu

CASES = [dict(n=5, n_gs=2, lgs=True, n_layer=3, seed=4, pad_L=12),
         dict(n=7, n_gs=3, lgs=True, n_layer=2, seed=5, pad_L=16)]


def _wl(case):
    return W.tiny(**case) if isinstance(case, dict) else case()


def _system(wl):
    from paper_1806_07938_amd import Context
    var, cxy = W.elongated_noise(wl)
    ctx = Context(0)
    k = ctx.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, wl.h_lgs, wl.gs, wl.valid, wl.h, wl.w, wl.r0, wl.L0)
    ctx.set_system(k, noise_var=var)
    ctx.set_noise_xy(cxy)
    return ctx, k, var, cxy


@pytest.mark.parametrize("case", CASES + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_products_with_2x2_noise(case):
    import torch
    from oracle.covariance import system_matrix
    wl = _wl(case)
    ctx, k, var, cxy = _system(wl)
    A = system_matrix(wl, var, cxy)
    dev = torch_dev()
    x = np.random.default_rng(2).standard_normal(wl.n_slopes)
    assert rel_maxabs(ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy(), A @ x) < 1e-11
    x32 = x.astype(np.float32)
    assert rel_maxabs(ctx.matvec(torch.tensor(x32, device=dev)).cpu().numpy(), A @ x32.astype(np.float64)) < 3e-6
    # removing the blocks restores the diagonal system
    ctx.set_noise_xy(None)
    assert rel_maxabs(ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy(), system_matrix(wl, var) @ x) < 1e-11


SOLVES = [dict(solver=0, precision=0), dict(solver=0, precision=1), dict(solver=1, precision=0),
          dict(solver=0, precision=0, preconditioner=1), dict(solver=0, precision=0, method=1),
          dict(solver=0, precision=1, method=1)]


@pytest.mark.parametrize("opts", SOLVES, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()))
@pytest.mark.parametrize("case", CASES + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_solves_with_2x2_noise(case, opts):
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    wl = _wl(case)
    ctx, k, var, cxy = _system(wl)
    A = system_matrix(wl, var, cxy)
    s = (W.turbulent_slopes(wl, noise=False)[0] + W.correlated_noise(var, cxy)).astype(np.float32)
    s64 = s.astype(np.float64)
    tol = 1e-9
    z, _, info = ctx.solve(torch.tensor(s, device=torch_dev()), tol=tol, **opts)
    zz = z.cpu().numpy()
    res = np.linalg.norm(s64 - A @ zz) / np.linalg.norm(s64)
    zref = cholesky_solve(A, s64)
    say("noise2x2", wl.name, opts, "iterations", info.iterations, "residual", res)
    assert info.status == 0
    assert res <= 1.01 * tol
    assert np.linalg.norm(zz - zref) <= 1e-5 * np.linalg.norm(zref)


def test_2x2_noise_errors():
    import torch
    from paper_1806_07938_amd import Context, TTError
    from paper_1806_07938_amd.tt import TT_INVALID_ARG, TT_NOT_READY
    wl = W.lgs3_10x10()
    ctx = Context(0)
    with pytest.raises(TTError) as e:
        ctx.set_noise_xy(np.zeros((wl.n_gs, 76)))
    assert e.value.status == TT_NOT_READY
    ctx2, k, var, cxy = _system(wl)
    bad = cxy.copy()
    bad[0, 0] = 2.0 * np.sqrt(var[0] * var[76])          # |cov| above sqrt(var_x var_y)
    with pytest.raises(TTError) as e:
        ctx2.set_noise_xy(bad)
    assert e.value.status == TT_INVALID_ARG
    s = torch.ones(wl.n_slopes, dtype=torch.float32, device=torch_dev())
    with pytest.raises(TTError) as e:                    # FP64 preconditioned solver with 2x2 blocks
        ctx2.solve(s, precision=1, preconditioner=1)
    assert e.value.status == TT_INVALID_ARG
