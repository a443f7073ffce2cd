"""Batched products and batched solves on uneven systems (grids 40 / 60 / 74 /
84, 4-8 LGS, 10-35 layers, noise 0.01-0.5 rad^2, L = 128 or 256), through the
C ABI, against the oracle's FP64 step-by-step 2RBT operator of each system
(itself pinned to the dense product on small grids).

Products: 3e-6 of the largest entry (FP32 spectra and transforms).  Solves
(batched CG and batched PCG, one measured frame per system): every frame
certified by the library's FP64 residual, and the residual recomputed with
the oracle's operator within 1.01 x tol."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uneven():
    from oracle.covariance import kernel_tables
    from oracle.toeplitz import ToeplitzOperator
    wls = [W.uneven_family(i) for i in range(4)]
    say("uneven systems:", [wl.name for wl in wls])
    systems = [make_system(wl, target=False) for wl in wls]
    workers = min(16, os.cpu_count() or 1)
    say("uneven systems: oracle tables with", workers, "workers")
    ops = [ToeplitzOperator(wl, tables=kernel_tables(wl, workers=workers)) for wl in wls]
    return wls, systems, ops


def test_uneven_batched_product(uneven):
    import torch
    from paper_1806_07938_amd import matvec_batch
    wls, systems, ops = uneven
    dev = torch_dev()
    rng = np.random.default_rng(21)
    xs = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    ys = matvec_batch([c for c, k in systems], [torch.tensor(x, device=dev) for x in xs])
    for wl, op, x, y in zip(wls, ops, xs, ys):
        assert rel_maxabs(y.cpu().numpy(), op(x.astype(np.float64))) < 3e-6, wl.name


@pytest.mark.parametrize("pc", [0, 1], ids=["cg", "pcg"])
def test_uneven_batched_solves(uneven, pc):
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED
    wls, systems, ops = uneven
    dev = torch_dev()
    S = [W.turbulent_slopes(wl)[0].astype(np.float32) for wl in wls]
    tol = 1e-6
    zs, _, infos, st = solve_batch([c for c, k in systems], [torch.tensor(s, device=dev) for s in S], tol=tol,
                                   solver=SOLVER_BATCHED, preconditioner=pc)
    assert st == 0
    for wl, op, s, z, inf in zip(wls, ops, S, zs, infos):
        say("uneven", "pcg" if pc else "cg", wl.name, "iterations", inf.iterations, "rel", inf.rel_residual)
        assert inf.status == 0 and inf.rel_residual <= tol
        sd = s.astype(np.float64)
        assert np.linalg.norm(sd - op(z.cpu().numpy())) <= 1.01 * tol * np.linalg.norm(sd), wl.name


# Half-precision spectra storage (tt_matvec_batch_prec).  Each frequency's
# stored values carry an absolute rounding error of at most u times that
# frequency's largest value (FP16, scaled to [2^14, 2^15): u = 2^-11; BF16:
# u = 2^-8), so by Parseval the product error is bounded in 2-norm by
# C u ||A||_2 ||x||_2 (C channels; a frequency's C x C block has norm <= C times
# its largest entry, which is <= ||A||_2).  ||A||_2 is under-estimated here by
# power iteration, which only tightens the check.
HALF_FORMS = {2: 2.0 ** -11, 3: 2.0 ** -8}


def _norm_estimate(op, n, rng, its=30):
    v = rng.standard_normal(n)
    lam = 0.0
    for _ in range(its):
        w = op(v)
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return lam


@pytest.mark.parametrize("precision", sorted(HALF_FORMS), ids=["f16", "bf16"])
def test_uneven_batched_product_half_spectra(uneven, precision):
    import torch
    from paper_1806_07938_amd import matvec_batch
    wls, systems, ops = uneven
    dev = torch_dev()
    rng = np.random.default_rng(23)
    xs = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    ys = matvec_batch([c for c, k in systems], [torch.tensor(x, device=dev) for x in xs], precision=precision)
    u = HALF_FORMS[precision]
    for wl, op, x, y in zip(wls, ops, xs, ys):
        ref = op(x.astype(np.float64))
        err = np.linalg.norm(y.cpu().numpy() - ref)
        bound = 2 * wl.n_gs * u * _norm_estimate(op, wl.n_slopes, rng) * np.linalg.norm(x)
        say(f"{wl.name} precision {precision}: |dy| / (C u |A| |x|) = {err / bound:.3e}, "
            f"rel max-abs {rel_maxabs(y.cpu().numpy(), ref):.2e}")
        assert err <= bound


@pytest.mark.parametrize("precision", sorted(HALF_FORMS), ids=["f16", "bf16"])
def test_uneven_batched_pcg_half_spectra(uneven, precision):
    """Batched PCG whose block-circulant preconditioner streams FP16 / BF16
    spectra: the product stays FP32, so every frame still reaches the
    tolerance, certified by the FP64 residual and by the oracle's operator."""
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import PRECOND_CIRCULANT, SOLVER_BATCHED
    wls, systems, ops = uneven
    dev = torch_dev()
    S = [W.turbulent_slopes(wl)[0].astype(np.float32) for wl in wls]
    tol = 1e-6
    zs, _, infos, st = solve_batch([c for c, k in systems], [torch.tensor(s, device=dev) for s in S], tol=tol,
                                   solver=SOLVER_BATCHED, preconditioner=PRECOND_CIRCULANT, precision=precision)
    assert st == 0
    for wl, op, s, z, inf in zip(wls, ops, S, zs, infos):
        zz = z.cpu().numpy()
        res = np.linalg.norm(s - op(zz)) / np.linalg.norm(s)
        say("uneven pcg precision", precision, wl.name, "iterations", inf.iterations, "rel", inf.rel_residual,
            "oracle", res)
        assert inf.status == 0 and inf.rel_residual <= tol and res <= 1.01 * tol


def test_uneven_64_system_batch(uneven):
    """64 uneven systems (uneven_family 0..63: grids 40 / 60 / 74 / 84, 4-8 LGS,
    10-35 layers) solved together by lockstep plain CG: every frame certified by
    its FP64 true residual, and the first four (the systems the oracle operators
    of this module belong to) by the oracle's operator.  Right-hand sides are
    seeded white noise (the solver's correctness does not depend on their
    statistics; the benchmark uses measured frames).  The least damped system
    (uneven_62: 8 LGS, noise variance 0.016 rad^2) needs 11-20 thousand plain-CG
    iterations for such right-hand sides, a count that moves by thousands with
    the rounding of the FP32 product, so the cap is well above it."""
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED
    wls4, systems4, ops = uneven
    dev = torch_dev()
    wls = wls4 + [W.uneven_family(i) for i in range(4, 64)]
    systems = systems4 + [make_system(wl, target=False) for wl in wls[4:]]
    rng = np.random.default_rng(64)
    S = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    tol = 1e-6
    zs, _, infos, st = solve_batch([c for c, k in systems], [torch.tensor(s, device=dev) for s in S], tol=tol,
                                   solver=SOLVER_BATCHED, max_iter=60000)
    its = [inf.iterations for inf in infos]
    say(f"64 uneven systems: status {st}, iterations {min(its)}-{max(its)}, max rel residual "
        f"{max(inf.rel_residual for inf in infos):.2e}")
    assert st == 0
    assert all(inf.status == 0 and inf.rel_residual <= tol for inf in infos)
    for op, s, z in zip(ops, S[:4], zs[:4]):
        res = np.linalg.norm(s - op(z.cpu().numpy())) / np.linalg.norm(s)
        assert res <= 1.01 * tol
    for c, k in systems[4:]:
        c.close()
        k.close()


@pytest.mark.parametrize("split", [1, 2, 4])
def test_uneven_batched_product_every_split(uneven, split):
    """The column kernel with each frequency split (S = 1: whole columns, 2, 4:
    folded columns, L / 4 < n for some systems) against the oracle operators."""
    import torch
    from paper_1806_07938_amd import matvec_batch
    wls, systems, ops = uneven
    dev = torch_dev()
    rng = np.random.default_rng(31 + split)
    xs = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    ys = matvec_batch([c for c, k in systems], [torch.tensor(x, device=dev) for x in xs], split=split)
    for wl, op, x, y in zip(wls, ops, xs, ys):
        err = rel_maxabs(y.cpu().numpy(), op(x.astype(np.float64)))
        say(f"split {split} {wl.name}: rel max-abs {err:.2e}")
        assert err < 3e-6, wl.name


def test_tuned_split_is_used_and_exact(uneven):
    import torch
    from paper_1806_07938_amd import matvec_batch
    from paper_1806_07938_amd.tt import tune_batch
    wls, systems, ops = uneven
    ctxs = [c for c, k in systems]
    best, ms = tune_batch(ctxs, op=0)
    say(f"tuned split {best}, ms per split {ms}")
    assert best in (1, 2, 4) and ms[best] is not None and ms[best] == min(v for v in ms.values() if v)
    dev = torch_dev()
    rng = np.random.default_rng(41)
    xs = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    ys = matvec_batch(ctxs, [torch.tensor(x, device=dev) for x in xs])
    for op, x, y in zip(ops, xs, ys):
        assert rel_maxabs(y.cpu().numpy(), op(x.astype(np.float64))) < 3e-6
