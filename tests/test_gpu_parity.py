"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes span several tiles and ragged tails (odd and even padding, random
masks, one to four guide stars, NGS and LGS) and the 10x10 / 3 LGS workload.
Tolerances: FP64 results to 1e-11 of the largest entry (two independent FP64
Bessel implementations, second differences of D); FP32 matrix-vector
products to 3e-6 of the largest entry (FP32 spectra and transforms); FP32
solves certified by the library's FP64 residual and checked against the
Cholesky solution to 1e-5 relative (the bound the method's FP32 path is held
to); projections to 1e-5 relative."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, oracle_tables_packed, rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu

TINY = [
    dict(n=1, n_gs=1, lgs=False, n_layer=1, seed=0, mask="full"),
    dict(n=2, n_gs=1, lgs=True, n_layer=2, seed=1, mask="full"),
    dict(n=3, n_gs=2, lgs=True, n_layer=2, seed=2),
    dict(n=4, n_gs=3, lgs=False, n_layer=3, seed=3),
    dict(n=5, n_gs=2, lgs=True, n_layer=4, seed=4, pad_L=12),
    dict(n=7, n_gs=4, lgs=True, n_layer=2, seed=5, pad_L=16),
    dict(n=8, n_gs=2, lgs=True, n_layer=3, seed=6, pad_L=19),
]


def _wl(case):
    return W.tiny(**case) if isinstance(case, dict) else case()


@pytest.mark.parametrize("case", TINY + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_kernel_tables(case):
    wl = _wl(case)
    say("tables", wl.name, "n", wl.n, "gs", wl.n_gs)
    ctx, k = make_system(wl, target=False)
    got = k.tables()
    ref = oracle_tables_packed(wl)
    assert got.shape == ref.shape
    assert rel_maxabs(got, ref) < 1e-11


@pytest.mark.parametrize("case", TINY + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_matvec(case):
    import torch
    from oracle.covariance import system_matrix
    wl = _wl(case)
    say("matvec", wl.name, "L", wl.pad_L)
    dev = torch_dev()
    ctx, k = make_system(wl, target=False)
    A = system_matrix(wl)
    rng = np.random.default_rng(11)
    for trial in range(2):
        x = rng.standard_normal(wl.n_slopes)
        x32 = x.astype(np.float32)
        y64 = ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy()
        assert rel_maxabs(y64, A @ x) < 1e-11
        y32 = ctx.matvec(torch.tensor(x32, device=dev)).cpu().numpy()
        assert rel_maxabs(y32, A @ x32.astype(np.float64)) < 3e-6


@pytest.mark.parametrize("L", [19, 20, 21, 32, 64])
def test_matvec_padding_invariance_10x10(L):
    import torch
    from oracle.covariance import system_matrix
    wl = W.lgs3_10x10(pad_L=L)
    say("matvec 10x10 L", L)
    dev = torch_dev()
    ctx, k = make_system(wl, target=False)
    x = np.random.default_rng(L).standard_normal(wl.n_slopes)
    y = ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy()
    assert rel_maxabs(y, system_matrix(wl) @ x) < 1e-11


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("solver", [1, 0])
def test_solve_10x10(precision, solver):
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    wl = W.lgs3_10x10()
    say("solve 10x10 precision", precision, "solver", solver)
    dev = torch_dev()
    ctx, k = make_system(wl, target=True)
    s = W.turbulent_slopes(wl)[0].astype(np.float32)
    A = system_matrix(wl)
    zref = cholesky_solve(A, s.astype(np.float64))
    zeta, phi, info = ctx.solve(torch.tensor(s, device=dev), tol=1e-10, precision=precision, solver=solver)
    z = zeta.cpu().numpy()
    say("  iters", info.iterations, "refinements", info.refinements, "relres", info.rel_residual)
    res = np.linalg.norm(s - A @ z) / np.linalg.norm(s)
    assert res <= 1.01e-10
    assert info.rel_residual <= 1e-10
    assert abs(info.rel_residual - res) <= 1e-11
    assert rel_maxabs(z, zref) < 1e-5


@pytest.mark.parametrize("case", TINY[2:] + [W.lgs3_10x10], ids=lambda c: str(c) if isinstance(c, dict) else "lgs3_10x10")
def test_projection(case):
    import torch
    from oracle.projection import phi_paper_dense
    wl = _wl(case)
    say("projection", wl.name)
    dev = torch_dev()
    ctx, k = make_system(wl, target=True)
    z = np.random.default_rng(3).standard_normal(wl.n_slopes)
    phi = ctx.project(torch.tensor(z, device=dev)).cpu().numpy()
    ref = phi_paper_dense(wl, z.astype(np.float32).astype(np.float64))
    assert phi.shape == ref.shape
    assert rel_maxabs(phi, ref) < 1e-5


@pytest.mark.parametrize("case", [dict(n=4, n_gs=3, lgs=True, n_layer=2, seed=3), dict(n=6, n_gs=2, lgs=False, n_layer=3, seed=8)])
def test_fried_model(case):
    # App. A.3 Fried gradient model: tables, matrix-vector product and projection
    import torch
    from oracle.covariance import system_matrix
    from oracle.projection import phi_paper_dense
    wl = W.tiny(**case)
    wl.model = "fried"
    say("fried", wl.name)
    dev = torch_dev()
    ctx, k = make_system(wl, target=True)
    assert rel_maxabs(k.tables(), oracle_tables_packed(wl)) < 1e-11
    x = np.random.default_rng(4).standard_normal(wl.n_slopes)
    assert rel_maxabs(ctx.matvec_f64(torch.tensor(x, device=dev)).cpu().numpy(), system_matrix(wl) @ x) < 1e-11
    phi = ctx.project(torch.tensor(x, device=dev)).cpu().numpy()
    ref = phi_paper_dense(wl, x.astype(np.float32).astype(np.float64))
    assert rel_maxabs(phi, ref) < 1e-5


def test_library_mask_rule_builds_the_same_system():
    # valid = NULL: the library's valid-subaperture rule with the obstruction
    # gives the workload's mask, hence the same tables, sizes and product
    import torch
    from paper_1806_07938_amd import Context
    wl = W.lgs3_10x10()
    say("library mask rule 10x10")
    dev = torch_dev()
    ctx, k = make_system(wl, target=False)
    c2 = Context(0)
    k2 = c2.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, wl.h_lgs, wl.gs, None, wl.h, wl.w, wl.r0, wl.L0,
                             obstruction=wl.obstruction)
    c2.set_system(k2, noise_scalar=wl.noise_var)
    assert c2.info["n_vs"] == 76 and c2.info["n_slopes"] == 456
    assert np.array_equal(k2.tables(), k.tables())
    x = torch.tensor(np.random.default_rng(2).standard_normal(wl.n_slopes), device=dev)
    assert torch.equal(c2.matvec_f64(x), ctx.matvec_f64(x))
    c2.close()
    k2.close()
    ctx.close()
    k.close()


def test_persistent_solver_refuses_more_columns_than_compute_units():
    # pad_L / 2 + 1 frequency columns beyond the compute units: the persistent
    # solver refuses before launching; the one-launch-per-phase solver solves
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    from paper_1806_07938_amd.tt import SOLVER_KERNELS, TT_INVALID_ARG, TTError
    wl = W.tiny(n=4, n_gs=2, lgs=True, n_layer=2, seed=5, pad_L=1022)
    say("pad_L 1022 persistent refusal")
    dev = torch_dev()
    ctx, k = make_system(wl, target=False)
    s = torch.tensor(W.gaussian_slopes(wl)[0].astype(np.float32), device=dev)
    with pytest.raises(TTError) as e:
        ctx.solve(s, tol=1e-8)
    assert e.value.status == TT_INVALID_ARG
    zeta, _, info = ctx.solve(s, tol=1e-8, solver=SOLVER_KERNELS)
    zref = cholesky_solve(system_matrix(wl), s.cpu().numpy().astype(np.float64))
    assert info.status == 0 and rel_maxabs(zeta.cpu().numpy(), zref) < 1e-5
    ctx.close()
    k.close()
