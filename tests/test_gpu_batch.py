"""tt_solve_batch through the C ABI: a batch of frames on systems of different
sizes and geometries (one context each) gives, frame by frame, the results of
tt_solve_frame (bitwise: the same deterministic kernels run), reaches each
oracle solution, and reports per-frame info and the worst status."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, say, torch_dev

pytestmark = pytest.mark.gpu


def _batch():
    wls = [W.lgs3_10x10(), W.tiny(n=6, n_gs=2, lgs=True, n_layer=3, seed=4, pad_L=12),
           W.tiny(n=8, n_gs=4, lgs=False, n_layer=2, seed=6, pad_L=16)]
    systems = [make_system(wl, target=True) for wl in wls]
    return wls, systems


def test_batch_equals_single_frames_and_oracle():
    import torch
    from oracle.covariance import system_matrix
    from oracle.solve import cholesky_solve
    from paper_1806_07938_amd import solve_batch
    wls, systems = _batch()
    dev = torch_dev()
    S = [torch.tensor(W.turbulent_slopes(wl)[0].astype(np.float32), device=dev) for wl in wls]
    ctxs = [c for c, k in systems]
    zs, phis, infos, st = solve_batch(ctxs, S, tol=1e-9)
    assert st == 0
    for wl, ctx, s, z, ph, inf in zip(wls, ctxs, S, zs, phis, infos):
        z1, ph1, inf1 = ctx.solve(s, tol=1e-9)
        say("batch", wl.name, "iterations", inf.iterations, inf1.iterations)
        assert np.array_equal(z.cpu().numpy(), z1.cpu().numpy())
        assert np.array_equal(ph.cpu().numpy(), ph1.cpu().numpy())
        assert inf.iterations == inf1.iterations and inf.status == 0
        A = system_matrix(wl)
        zref = cholesky_solve(A, s.cpu().numpy().astype(np.float64))
        assert np.linalg.norm(z.cpu().numpy() - zref) <= 1e-5 * np.linalg.norm(zref)


def test_batch_status_and_errors():
    import torch
    from paper_1806_07938_amd import TTError, solve_batch
    from paper_1806_07938_amd.tt import TT_INVALID_ARG, TT_NOT_CONVERGED
    wls, systems = _batch()
    dev = torch_dev()
    ctxs = [c for c, k in systems]
    S = [torch.tensor(W.turbulent_slopes(wl)[0].astype(np.float32), device=dev) for wl in wls]
    # a cap that stops every frame: all frames attempted, worst status returned
    zs, phis, infos, st = solve_batch(ctxs, S, tol=1e-12, max_iter=3, allow=(0, TT_NOT_CONVERGED))
    assert st == TT_NOT_CONVERGED and all(i.status == TT_NOT_CONVERGED and i.iterations == 3 for i in infos)
    with pytest.raises(TTError) as e:
        solve_batch([ctxs[0], ctxs[0]], [S[0], S[0]])
    assert e.value.status == TT_INVALID_ARG
    zs, phis, infos, st = solve_batch([], [])
    assert st == 0 and zs == []
