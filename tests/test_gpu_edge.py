"""Edge cases and failure handling of the HIP path through the C ABI: iteration
caps, zero tolerance, zero input, warm start, breakdown (NaN input, an
indefinite system forced from the host through the noise variance), per-slope
noise, natural guide stars, an off-axis target, and argument / state errors.
Every failure is forced from the host; every kernel still exits normally."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu

SOLVERS = [0, 1]


@pytest.fixture(scope="module")
def c1sys():
    wl = W.lgs3_10x10()
    ctx, k = make_system(wl, target=True)
    return wl, ctx, k


def _s(wl, seed=3):
    return W.turbulent_slopes(wl, seed=seed)[0].astype(np.float32)


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("precision", [0, 1])
def test_iteration_cap(c1sys, solver, precision):
    import torch
    from paper_1806_07938_amd.tt import TT_NOT_CONVERGED
    wl, ctx, k = c1sys
    say("cap solver", solver, "precision", precision)
    s = torch.tensor(_s(wl), device=torch_dev())
    for cap in (0, 1, 7):
        z, phi, info = ctx.solve(s, tol=1e-10, max_iter=cap, solver=solver, precision=precision,
                                 allow=(0, TT_NOT_CONVERGED))
        assert info.status == TT_NOT_CONVERGED
        assert info.iterations == cap
        assert np.all(np.isfinite(z.cpu().numpy()))
        assert 0 < info.rel_residual <= 1.0 + 1e-12


@pytest.mark.parametrize("solver", SOLVERS)
def test_zero_tolerance_hits_cap(c1sys, solver):
    import torch
    from paper_1806_07938_amd.tt import TT_NOT_CONVERGED
    wl, ctx, k = c1sys
    s = torch.tensor(_s(wl), device=torch_dev())
    z, phi, info = ctx.solve(s, tol=0.0, max_iter=40, solver=solver, allow=(0, TT_NOT_CONVERGED))
    assert info.status == TT_NOT_CONVERGED and info.iterations == 40


@pytest.mark.parametrize("solver", SOLVERS)
def test_zero_slopes(c1sys, solver):
    import torch
    wl, ctx, k = c1sys
    s = torch.zeros(wl.n_slopes, dtype=torch.float32, device=torch_dev())
    z, phi, info = ctx.solve(s, solver=solver)
    assert info.status == 0 and info.iterations == 0
    assert np.all(z.cpu().numpy() == 0) and np.all(phi.cpu().numpy() == 0)


@pytest.mark.parametrize("solver", SOLVERS)
def test_warm_start_at_solution(c1sys, solver):
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    wl, ctx, k = c1sys
    s = _s(wl)
    zref = cholesky_solve(system_matrix(wl), s.astype(np.float64))
    dev = torch_dev()
    z, phi, info = ctx.solve(torch.tensor(s, device=dev), x0=torch.tensor(zref, device=dev), tol=1e-6, solver=solver)
    assert info.status == 0 and info.iterations == 0
    assert np.linalg.norm(z.cpu().numpy() - zref) <= 1e-12 * np.linalg.norm(zref)


@pytest.mark.parametrize("solver", SOLVERS)
def test_warm_start_from_previous_frame_saves_iterations(c1sys, solver):
    import torch
    wl, ctx, k = c1sys
    dev = torch_dev()
    s = W.turbulent_slopes(wl, seed=4, frames=1)[0].astype(np.float32)
    z0, _, i0 = ctx.solve(torch.tensor(s, device=dev), tol=1e-8, solver=solver)
    s2 = (s + 0.05 * np.random.default_rng(1).standard_normal(s.size)).astype(np.float32)
    _, _, cold = ctx.solve(torch.tensor(s2, device=dev), tol=1e-8, solver=solver)
    _, _, warm = ctx.solve(torch.tensor(s2, device=dev), x0=z0.clone(), tol=1e-8, solver=solver)
    assert warm.status == 0 and cold.status == 0
    assert warm.iterations < cold.iterations


@pytest.mark.parametrize("solver", SOLVERS)
def test_nan_input_is_breakdown(c1sys, solver):
    import torch
    from paper_1806_07938_amd.tt import TT_BREAKDOWN
    wl, ctx, k = c1sys
    s = _s(wl)
    s[5] = np.nan
    z, phi, info = ctx.solve(torch.tensor(s, device=torch_dev()), solver=solver, allow=(TT_BREAKDOWN,))
    assert info.status == TT_BREAKDOWN


@pytest.mark.parametrize("solver", SOLVERS)
def test_indefinite_system_is_breakdown(solver):
    # sigma^2 far below minus the largest covariance eigenvalue makes A negative
    # definite: p.Ap < 0 at the first iteration.
    import torch
    from paper_1806_07938_amd import Context, system_from
    from paper_1806_07938_amd.tt import TT_BREAKDOWN
    wl = W.lgs3_10x10()
    s = _s(wl)
    wl.noise_var = -1e5
    ctx = Context(0)
    system_from(ctx, wl, target=False)
    z, phi, info = ctx.solve(torch.tensor(s, device=torch_dev()), solver=solver, allow=(TT_BREAKDOWN,))
    assert info.status == TT_BREAKDOWN


@pytest.mark.parametrize("solver", SOLVERS)
def test_per_slope_noise(solver):
    import torch
    from oracle.covariance import slope_covariance
    from oracle.solve import cholesky_solve
    from paper_1806_07938_amd import Context
    wl = W.lgs3_10x10()
    nz = 0.05 + 0.3 * np.random.default_rng(2).random(wl.n_slopes)
    ctx = Context(0)
    k = ctx.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, wl.h_lgs, wl.gs, wl.valid, wl.h, wl.w, wl.r0, wl.L0)
    ctx.set_system(k, noise_var=nz)
    A = slope_covariance(wl) + np.diag(nz)
    s = _s(wl)
    dev = torch_dev()
    x = np.random.default_rng(0).standard_normal(wl.n_slopes)
    y = ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy()
    assert rel_maxabs(y, A @ x) < 1e-11
    z, _, info = ctx.solve(torch.tensor(s, device=dev), tol=1e-10, solver=solver)
    zref = cholesky_solve(A, s.astype(np.float64))
    assert np.linalg.norm(z.cpu().numpy() - zref) / np.linalg.norm(zref) < 1e-5


@pytest.mark.parametrize("solver", SOLVERS)
def test_ngs_and_off_axis_target(solver):
    import torch
    from oracle.covariance import system_matrix
    from oracle.projection import phi_exact, phi_paper_dense
    from oracle.solve import cholesky_solve
    wl = W.lgs3_10x10()
    wl.h_lgs = math.inf
    wl.target = (8 * W.ARCSEC, -5 * W.ARCSEC)
    ctx, k = make_system(wl, target=True)
    assert ctx.info["n_prime"] == wl.n + 1
    s = _s(wl)
    dev = torch_dev()
    z, phi, info = ctx.solve(torch.tensor(s, device=dev), tol=1e-10, solver=solver)
    zref = cholesky_solve(system_matrix(wl), s.astype(np.float64))
    assert np.linalg.norm(z.cpu().numpy() - zref) / np.linalg.norm(zref) < 1e-5
    ref = phi_paper_dense(wl, z.cpu().numpy().astype(np.float32).astype(np.float64))
    assert rel_maxabs(phi.cpu().numpy(), ref) < 1e-5
    # natural guide stars: the paper's grid form is the exact product
    ex = phi_exact(wl, z.cpu().numpy().astype(np.float32).astype(np.float64))
    assert np.linalg.norm(ref - ex) / np.linalg.norm(ex) < 1e-10


def test_argument_and_state_errors():
    import torch
    from paper_1806_07938_amd import Context, TTError
    from paper_1806_07938_amd.tt import TT_INVALID_ARG, TT_NOT_READY
    wl = W.lgs3_10x10()
    ctx = Context(0)
    dev = torch_dev()
    with pytest.raises(TTError) as e:
        ctx.generate_kernels(wl.n, wl.n_gs, 2 * wl.n - 2, wl.D, wl.h_lgs, wl.gs, wl.valid, wl.h, wl.w, wl.r0, wl.L0)
    assert e.value.status == TT_INVALID_ARG
    with pytest.raises(TTError) as e:
        ctx.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, 9e3, wl.gs, wl.valid, wl.h, wl.w, wl.r0, wl.L0)
    assert e.value.status == TT_INVALID_ARG          # layer above the LGS
    with pytest.raises(TTError) as e:
        ctx.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, wl.h_lgs, wl.gs, np.zeros_like(wl.valid), wl.h, wl.w,
                             wl.r0, wl.L0)
    assert e.value.status == TT_INVALID_ARG          # no valid subaperture
    from paper_1806_07938_amd import tt
    import ctypes as C
    zeta = torch.zeros(wl.n_slopes, dtype=torch.float64, device=dev)
    s = torch.zeros(wl.n_slopes, dtype=torch.float32, device=dev)
    st = tt.load().tt_solve_frame(ctx._h, C.c_void_p(s.data_ptr()), None, C.c_void_p(zeta.data_ptr()), None, None,
                                  None)
    assert st == TT_NOT_READY
    k = ctx.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, wl.h_lgs, wl.gs, wl.valid, wl.h, wl.w, wl.r0, wl.L0)
    ctx.set_system(k, noise_scalar=wl.noise_var)       # no target
    phi = torch.zeros(100, dtype=torch.float32, device=dev)
    st = tt.load().tt_solve_frame(ctx._h, C.c_void_p(s.data_ptr()), None, C.c_void_p(zeta.data_ptr()),
                                  C.c_void_p(phi.data_ptr()), None, None)
    assert st == TT_NOT_READY
    with pytest.raises(TTError) as e:
        ctx.solve(s, tol=-1.0)
    assert e.value.status == TT_INVALID_ARG


def test_two_systems_and_repeated_solves():
    # a context re-used for a second, smaller system; repeated solves agree
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    from paper_1806_07938_amd import Context, system_from
    ctx = Context(0)
    dev = torch_dev()
    for wl in (W.lgs3_10x10(), W.tiny(n=5, n_gs=2, seed=3, pad_L=10)):
        system_from(ctx, wl, target=True)
        s = W.gaussian_slopes(wl, seed=1)[0].astype(np.float32)
        zref = cholesky_solve(system_matrix(wl), s.astype(np.float64))
        z1, _, _ = ctx.solve(torch.tensor(s, device=dev), tol=1e-9)
        z2, _, _ = ctx.solve(torch.tensor(s, device=dev), tol=1e-9)
        assert np.linalg.norm(z1.cpu().numpy() - zref) / np.linalg.norm(zref) < 1e-5
        assert np.array_equal(z1.cpu().numpy(), z2.cpu().numpy())


@pytest.mark.parametrize("n_prime", [0, 13])
def test_ngs_projection_layers_summed(n_prime):
    # natural guide stars: the library sums the layer spectra (one inverse
    # transform); the oracle keeps one product per layer.  Default grid
    # (n' = n + 1, identity interpolation) and a larger grid (interpolated).
    import torch
    from oracle.projection import phi_exact, phi_paper_dense
    wl = W.tiny(n=6, n_gs=3, lgs=False, n_layer=4, seed=9, pad_L=11)
    wl.target = (4 * W.ARCSEC, 2 * W.ARCSEC)
    ctx, k = make_system(wl, target=True, n_prime=n_prime)
    z = np.random.default_rng(7).standard_normal(wl.n_slopes)
    phi = ctx.project(torch.tensor(z, device=torch_dev())).cpu().numpy()
    z32 = z.astype(np.float32).astype(np.float64)
    ref = phi_paper_dense(wl, z32, n_prime=(n_prime or None))
    say("ngs projection n'", ctx.info["n_prime"], "difference", np.linalg.norm(phi - ref) / np.linalg.norm(ref))
    assert rel_maxabs(phi, ref) < 1e-5
    if n_prime == 0:
        assert np.linalg.norm(ref - phi_exact(wl, z32)) / np.linalg.norm(ref) < 1e-10
