"""TT_SOLVER_BATCHED through tt_solve_batch: CG on every system of the call in
lockstep, products by the batched 2RBT product.  Each frame against its own
oracle: the Cholesky solution of the dense system (1e-5 relative, the bound
the FP32 path with FP64 residual replacement is held to), the FP64 residual
recomputed with the oracle's dense matrix (the tolerance is certified), and the
projection of the returned zeta by the oracle's dense paper-form projection
(1e-5 relative).  Systems differ in size, guide stars, noise and padding;
also the statuses when frames stop early, warm starts, a batch of one through
tt_solve_frame, and the argument errors."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu


def _systems(target=True):
    wls = [W.lgs3_10x10(), W.tiny(n=6, n_gs=2, lgs=True, n_layer=3, seed=4, pad_L=12),
           W.tiny(n=8, n_gs=4, lgs=False, n_layer=2, seed=6, pad_L=16), W.lgs3_10x10(pad_L=32),
           W.tiny(n=5, n_gs=3, lgs=True, n_layer=2, seed=7, pad_L=10)]
    return wls, [make_system(wl, target=target) for wl in wls]


def _check_frame(wl, s, z, tol, inf):
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    A = system_matrix(wl)
    sd = s.astype(np.float64)
    zref = cholesky_solve(A, sd)
    assert inf.status == 0, wl.name
    assert inf.rel_residual <= tol
    assert np.linalg.norm(sd - A @ z) <= 1.01 * tol * np.linalg.norm(sd), wl.name
    assert rel_maxabs(z, zref) <= 1e-5, wl.name


@pytest.mark.parametrize("pc", [0, 1], ids=["cg", "pcg"])
@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_batched_solver_matches_oracle(tol, pc):
    import torch
    from oracle.projection import phi_paper_dense
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED
    wls, systems = _systems()
    dev = torch_dev()
    S = [torch.tensor(W.turbulent_slopes(wl)[0].astype(np.float32), device=dev) for wl in wls]
    zs, phis, infos, st = solve_batch([c for c, k in systems], S, tol=tol, solver=SOLVER_BATCHED, preconditioner=pc)
    assert st == 0
    for wl, s, z, ph, inf in zip(wls, S, zs, phis, infos):
        say("batched", "pcg" if pc else "cg", wl.name, "L", wl.pad_L, "iterations", inf.iterations,
            "refinements", inf.refinements, "rel", inf.rel_residual)
        zc = z.cpu().numpy()
        _check_frame(wl, s.cpu().numpy(), zc, tol, inf)
        ref = phi_paper_dense(wl, zc.astype(np.float32).astype(np.float64))
        assert np.linalg.norm(ph.cpu().numpy() - ref) <= 1e-5 * np.linalg.norm(ref), wl.name


def test_batched_solver_warm_start_and_single():
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED
    wls, systems = _systems(target=False)
    dev = torch_dev()
    S = [torch.tensor(W.turbulent_slopes(wl, frames=2)[1].astype(np.float32), device=dev) for wl in wls]
    zs, _, infos, st = solve_batch([c for c, k in systems], S, tol=1e-8, solver=SOLVER_BATCHED)
    assert st == 0
    # warm start from the solutions: converged before any iteration
    import ctypes as C
    from paper_1806_07938_amd import tt
    m = len(wls)
    arr = C.c_void_p * m
    zs2 = [torch.empty_like(z) for z in zs]
    opts = tt._SolveOpts(1e-8, 20000, tt.PREC_F32, SOLVER_BATCHED, 1e-3, tt.PRECOND_NONE, tt.METHOD_CG)
    infos2 = (tt._SolveInfo * m)()
    st2 = tt.load().tt_solve_batch(arr(*[c._h for c, k in systems]), m, arr(*[s.data_ptr() for s in S]),
                                   arr(*[z.data_ptr() for z in zs]), arr(*[z.data_ptr() for z in zs2]), None,
                                   C.byref(opts), infos2)
    assert st2 == 0
    for i in range(m):
        assert infos2[i].iterations == 0 and infos2[i].status == 0
        assert np.allclose(zs2[i].cpu().numpy(), zs[i].cpu().numpy(), rtol=0, atol=0)
    # a batch of one through tt_solve_frame
    z1, _, inf1 = systems[0][0].solve(S[0], tol=1e-8, solver=SOLVER_BATCHED, project=False)
    _check_frame(wls[0], S[0].cpu().numpy(), z1.cpu().numpy(), 1e-8, inf1)


def test_batched_solver_statuses_and_errors():
    import torch
    from paper_1806_07938_amd import TTError, solve_batch
    from paper_1806_07938_amd.tt import (PREC_F64, PRECOND_CIRCULANT, SOLVER_BATCHED, TT_INVALID_ARG,
                                         TT_NOT_CONVERGED)
    wls, systems = _systems(target=False)
    dev = torch_dev()
    ctxs = [c for c, k in systems]
    S = [torch.tensor(W.turbulent_slopes(wl)[0].astype(np.float32), device=dev) for wl in wls]
    # an iteration cap stops every frame; all frames reported
    for pc in (0, PRECOND_CIRCULANT):
        zs, _, infos, st = solve_batch(ctxs, S, tol=1e-12, max_iter=5, solver=SOLVER_BATCHED, preconditioner=pc,
                                       allow=(0, TT_NOT_CONVERGED))
        assert st == TT_NOT_CONVERGED
        assert all(i.status == TT_NOT_CONVERGED and i.iterations == 5 for i in infos)
    # max_iter = 0: no iteration, zeta = 0 and the true residual of it
    zs, _, infos, st = solve_batch(ctxs, S, max_iter=0, solver=SOLVER_BATCHED, preconditioner=PRECOND_CIRCULANT,
                                   allow=(0, TT_NOT_CONVERGED))
    assert st == TT_NOT_CONVERGED
    assert all(i.iterations == 0 and abs(i.rel_residual - 1.0) < 1e-12 for i in infos)
    assert all(float(z.abs().max()) == 0.0 for z in zs)
    # the first system converged at the start (zero right-hand side): the others
    # iterate on the stream of the first system still iterating
    Z0 = [torch.zeros_like(S[0])] + S[1:]
    zs, _, infos, st = solve_batch(ctxs, Z0, tol=1e-8, solver=SOLVER_BATCHED, preconditioner=PRECOND_CIRCULANT)
    assert st == 0 and infos[0].iterations == 0
    for wl, s, z, inf in list(zip(wls, Z0, zs, infos))[1:]:
        _check_frame(wl, s.cpu().numpy(), z.cpu().numpy(), 1e-8, inf)
    # a zero right-hand side is solved by zeta = 0 without iterating
    Z = [torch.zeros_like(s) for s in S]
    zs, _, infos, st = solve_batch(ctxs[:2], Z[:2], solver=SOLVER_BATCHED)
    assert st == 0 and all(i.iterations == 0 for i in infos)
    assert all(float(z.abs().max()) == 0.0 for z in zs)
    for kw in (dict(precision=PREC_F64), dict(precision=PREC_F64, preconditioner=PRECOND_CIRCULANT)):
        with pytest.raises(TTError) as e:
            solve_batch(ctxs, S, solver=SOLVER_BATCHED, **kw)
        assert e.value.status == TT_INVALID_ARG
    with pytest.raises(TTError) as e:
        solve_batch([ctxs[0], ctxs[0]], [S[0], S[0]], solver=SOLVER_BATCHED)
    assert e.value.status == TT_INVALID_ARG
    ctxs[1].set_mode_removal(True)
    with pytest.raises(TTError) as e:
        solve_batch(ctxs[:2], S[:2], solver=SOLVER_BATCHED)
    assert e.value.status == TT_INVALID_ARG
    ctxs[1].set_mode_removal(False)


def test_batched_pcg_four_way_split():
    # every pad_L a multiple of 4: the preconditioner's column items take a
    # quarter of the frequencies each, m = L / 4 below n (folded input), in
    # plain sums (L = 12, 20) and FFTs (L = 16, 32)
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT, SOLVER_BATCHED
    wls = [W.lgs3_10x10(), W.tiny(n=6, n_gs=2, lgs=True, n_layer=3, seed=4, pad_L=12),
           W.tiny(n=8, n_gs=4, lgs=False, n_layer=2, seed=6, pad_L=16), W.lgs3_10x10(pad_L=32)]
    systems = [make_system(wl, target=False) for wl in wls]
    dev = torch_dev()
    S = [torch.tensor(W.turbulent_slopes(wl)[0].astype(np.float32), device=dev) for wl in wls]
    zs, _, infos, st = solve_batch([c for c, k in systems], S, tol=1e-8, solver=SOLVER_BATCHED,
                                   preconditioner=PRECOND_CIRCULANT)
    assert st == 0
    for wl, s, z, inf in zip(wls, S, zs, infos):
        say("batched pcg, four-way split", wl.name, "L", wl.pad_L, "iterations", inf.iterations)
        _check_frame(wl, s.cpu().numpy(), z.cpu().numpy(), 1e-8, inf)


def test_views_solve_many_frames_of_one_system():
    """Several right-hand sides of one system (context views sharing its
    spectra) solved together by the batched solver: every frame certified by
    the oracle's dense residual, and equal to the same frame solved alone by
    the batched solver on the base context (the systems of a lockstep batch
    do not interact: bitwise equal)."""
    import torch
    from oracle.covariance import system_matrix
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT, SOLVER_BATCHED, TTError
    wl = W.lgs3_10x10()
    base, k = make_system(wl, target=True)
    views = [base.view() for _ in range(5)]
    frames = W.turbulent_slopes(wl, seed=77, frames=6).astype(np.float32)
    dev = torch_dev()
    S = [torch.tensor(f, device=dev) for f in frames]
    A = system_matrix(wl)
    for pc in (0, PRECOND_CIRCULANT):
        zs, phis, infos, st = solve_batch([base] + views, S, tol=1e-8, solver=SOLVER_BATCHED, preconditioner=pc)
        assert st == 0 and all(p is None for p in phis)
        for i, (f, z, inf) in enumerate(zip(frames, zs, infos)):
            zz = z.cpu().numpy()
            res = np.linalg.norm(f - A @ zz) / np.linalg.norm(f)
            say(f"view {i} pc {pc}: {inf.iterations} iterations, oracle residual {res:.2e}")
            assert inf.status == 0 and res <= 1.01e-8
            z1, _, inf1 = views[0].solve(S[i], tol=1e-8, solver=SOLVER_BATCHED, preconditioner=pc, project=False) \
                if i else base.solve(S[i], tol=1e-8, solver=SOLVER_BATCHED, preconditioner=pc, project=False)
            assert np.array_equal(z1.cpu().numpy(), zz) and inf1.iterations == inf.iterations
    # the base cannot change or go away while views share its system
    with pytest.raises(TTError):
        base.close()
    with pytest.raises(TTError):
        base.set_mode_removal(True)
    for v in views:
        v.close()
    base.close()
    k.close()


@pytest.mark.parametrize("pc", [0, 1, 2], ids=["cg", "circulant", "learned"])
def test_graph_replayed_chunks_equal_eager_launches(pc):
    """opts.graph: the lockstep chunks replayed from a captured HIP graph give
    bitwise the results of launching the same kernels one by one (many replays
    per solve, with the solver's own synchronisations between them), for plain
    CG, the block-circulant PCG and flexible CG with a learned network."""
    import torch
    from paper_1806_07938_amd import Learned, solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED
    wls = [W.lgs3_10x10(), W.lgs3_10x10_family(0), W.lgs3_10x10_family(1)]
    systems = [make_system(wl, target=False) for wl in wls]
    ctxs = [c for c, k in systems]
    net = None
    if pc == 2:
        net = Learned(3, 32, seed=5)
        net.train(ctxs, n_pairs=2000, steps=200, batch=8, lr=3e-3)
        for c in ctxs:
            c.set_learned(net)
    dev = torch_dev()
    S = [torch.tensor(W.turbulent_slopes(wl, seed=9)[0].astype(np.float32), device=dev) for wl in wls]
    ze, _, ie, st_e = solve_batch(ctxs, S, tol=1e-9, solver=SOLVER_BATCHED, preconditioner=pc)
    zg, _, ig, st_g = solve_batch(ctxs, S, tol=1e-9, solver=SOLVER_BATCHED, preconditioner=pc, graph=True)
    assert st_e == st_g == 0
    for a, b, x, y in zip(ze, zg, ie, ig):
        say(f"pc {pc}: eager {x.iterations} iterations, graph {y.iterations}")
        assert x.iterations == y.iterations and x.iterations > 3 * 16
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    for c, k in systems:
        c.close()
        k.close()
    if net is not None:
        net.close()
