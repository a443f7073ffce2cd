"""tt_matvec_batch: the FP32 2RBT product of many independent systems in one
call, each result against the FP64 oracle of its own system (the dense
definition on small systems, the oracle's step-by-step 2RBT evaluation at
74x74), through the C ABI.

Batches mix sizes, guide-star counts, masks and paddings so that both column
paths run: pad_L / S a power of two (radix-2 FFT) and not (plain sums), with
S = 2 (every pad_L even) and S = 1 (some pad_L odd).  Tolerance: 3e-6 of the
largest entry, as for the single-system FP32 product (FP32 spectra and
transforms)."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, rel_maxabs, say, torch_dev

pytestmark = pytest.mark.gpu

# pad_L odd somewhere: S = 1 (columns of 19, 21, 13 ... points)
ODD = [dict(n=1, n_gs=1, lgs=False, n_layer=1, seed=0, mask="full"),
       dict(n=3, n_gs=2, lgs=True, n_layer=2, seed=2),
       dict(n=8, n_gs=2, lgs=True, n_layer=3, seed=6, pad_L=19),
       dict(n=7, n_gs=4, lgs=True, n_layer=2, seed=5, pad_L=16),
       ("lgs3_10x10", 21), ("lgs3_10x10", 32)]
# every pad_L even: S = 2; pad_L / 2 = 6, 8, 10, 16, 32, 9
EVEN = [dict(n=5, n_gs=2, lgs=True, n_layer=4, seed=4, pad_L=12),
        dict(n=7, n_gs=4, lgs=True, n_layer=2, seed=5, pad_L=16),
        dict(n=2, n_gs=1, lgs=True, n_layer=2, seed=1, mask="full", pad_L=4),
        ("lgs3_10x10", 20), ("lgs3_10x10", 32), ("lgs3_10x10", 64),
        dict(n=4, n_gs=3, lgs=False, n_layer=3, seed=3, pad_L=18)]


def _wl(case):
    if isinstance(case, tuple):
        return W.lgs3_10x10(pad_L=case[1])
    return W.tiny(**case)


def _batch(cases, seed):
    import torch
    from oracle.covariance import system_matrix
    dev = torch_dev()
    wls = [_wl(c) for c in cases]
    systems = [make_system(wl, target=False) for wl in wls]
    rng = np.random.default_rng(seed)
    xs = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    refs = [system_matrix(wl) @ x.astype(np.float64) for wl, x in zip(wls, xs)]
    xd = [torch.tensor(x, device=dev) for x in xs]
    return wls, systems, xd, refs


@pytest.mark.parametrize("cases", [ODD, EVEN], ids=["S1", "S2"])
def test_batch_matches_oracle(cases):
    from paper_1806_07938_amd import matvec_batch
    wls, systems, xd, refs = _batch(cases, 3)
    say("matvec batch", [wl.name + f"/L{wl.pad_L}" for wl in wls])
    ys = matvec_batch([s[0] for s in systems], xd)
    for wl, y, ref in zip(wls, ys, refs):
        assert rel_maxabs(y.cpu().numpy(), ref) < 3e-6, wl.name
    # again in another order, with timing: descriptors rebuilt, same results
    order = list(reversed(range(len(wls))))
    ys2, ms = matvec_batch([systems[i][0] for i in order], [xd[i] for i in order], timing=True)
    assert len(ms) == 3 and all(v > 0 for v in ms)
    for j, i in enumerate(order):
        assert rel_maxabs(ys2[j].cpu().numpy(), refs[i]) < 3e-6, wls[i].name


def test_batch_subsets_and_single():
    from paper_1806_07938_amd import matvec_batch
    wls, systems, xd, refs = _batch(EVEN, 4)
    say("matvec batch subsets")
    for idx in ([0], [3, 1], [5, 2, 6]):
        ys = matvec_batch([systems[i][0] for i in idx], [xd[i] for i in idx])
        for y, i in zip(ys, idx):
            assert rel_maxabs(y.cpu().numpy(), refs[i]) < 3e-6
    assert matvec_batch([], []) == []


def test_batch_with_2x2_noise():
    import torch
    from oracle.covariance import system_matrix
    from paper_1806_07938_amd import Context, matvec_batch
    dev = torch_dev()
    say("matvec batch with 2x2 noise blocks")
    ctxs, refs, xd = [], [], []
    rng = np.random.default_rng(6)
    l256 = dict(n=7, n_gs=4, lgs=True, n_layer=2, seed=8, pad_L=256)   # the packed-channel L = 256 row transforms
    for case, xy in ((EVEN[0], True), (("lgs3_10x10", 20), True), (EVEN[1], False), (l256, True)):
        wl = _wl(case)
        var, cxy = W.elongated_noise(wl)
        ctx = Context(0)
        k = ctx.generate_kernels(wl.n, wl.n_gs, wl.pad_L, wl.D, wl.h_lgs, wl.gs, wl.valid, wl.h, wl.w, wl.r0, wl.L0)
        ctx.set_system(k, noise_var=var)
        if xy:
            ctx.set_noise_xy(cxy)
        x = rng.standard_normal(wl.n_slopes).astype(np.float32)
        refs.append(system_matrix(wl, var, cxy if xy else None) @ x.astype(np.float64))
        ctxs.append((ctx, k))
        xd.append(torch.tensor(x, device=dev))
    ys = matvec_batch([c[0] for c in ctxs], xd)
    for y, ref in zip(ys, refs):
        assert rel_maxabs(y.cpu().numpy(), ref) < 3e-6


def test_batch_argument_errors():
    import torch
    from paper_1806_07938_amd import TTError, matvec_batch, tt
    wls, systems, xd, refs = _batch(EVEN[:2], 5)
    a, b = systems[0][0], systems[1][0]
    with pytest.raises(TTError) as e:
        matvec_batch([a, a], [xd[0], xd[0]])
    assert e.value.status == tt.TT_INVALID_ARG
    b.set_mode_removal(True)
    with pytest.raises(TTError) as e:
        matvec_batch([a, b], xd)
    assert e.value.status == tt.TT_INVALID_ARG
    b.set_mode_removal(False)
    y = torch.empty_like(xd[0])
    with pytest.raises(TTError) as e:
        matvec_batch([a], [xd[0]], ys=[xd[0]])
    assert e.value.status == tt.TT_INVALID_ARG
    ys = matvec_batch([a, b], xd, ys=[y, torch.empty_like(xd[1])])
    assert ys[0] is y
    assert rel_maxabs(y.cpu().numpy(), refs[0]) < 3e-6


@pytest.fixture(scope="module")
def family74():
    """Two distinct 74x74 / 6 LGS systems at L = 256 (the benchmark's batch
    shape) and lgs6_74x74 at L = 148, with the oracle's FP64 2RBT operators."""
    from oracle.covariance import kernel_tables
    from oracle.toeplitz import ToeplitzOperator
    import os
    wls = [W.lgs6_74x74_family(0), W.lgs6_74x74_family(1), W.lgs6_74x74_family(-1, pad_L=148)]
    say("74x74 family: library systems")
    systems = [make_system(wl, target=False) for wl in wls]
    workers = min(16, os.cpu_count() or 1)
    say("74x74 family: oracle tables with", workers, "workers")
    ops = [ToeplitzOperator(wl, tables=kernel_tables(wl, workers=workers)) for wl in wls]
    return wls, systems, ops


def test_batch_74x74(family74):
    import torch
    from paper_1806_07938_amd import matvec_batch
    wls, systems, ops = family74
    dev = torch_dev()
    rng = np.random.default_rng(9)
    xs = [rng.standard_normal(wl.n_slopes).astype(np.float32) for wl in wls]
    say("74x74 batch: L = 256 (FFT columns) x2 and L = 148 (plain sums)")
    ys, ms = matvec_batch([s[0] for s in systems], [torch.tensor(x, device=dev) for x in xs], timing=True)
    say("phase ms", ms)
    for wl, op, x, y in zip(wls, ops, xs, ys):
        assert rel_maxabs(y.cpu().numpy(), op(x.astype(np.float64))) < 3e-6, wl.name


@pytest.mark.parametrize("cases", [
    # G = 4 at L = 256 next to G = 3: float loads, 6144 spectra floats per item (two rounds)
    [dict(n=7, n_gs=4, lgs=True, n_layer=2, seed=8, pad_L=256), ("lgs3_10x10", 20)],
    # G = 8 at L = 256: float4 loads, 24576 floats per item (two rounds), 117 KB of LDS per item
    [dict(n=3, n_gs=8, lgs=True, n_layer=2, seed=9, mask="full", pad_L=256),
     dict(n=4, n_gs=2, lgs=False, n_layer=2, seed=10, pad_L=8)],
], ids=["float", "float4"])
def test_batch_spectra_in_several_rounds(cases):
    from paper_1806_07938_amd import matvec_batch
    wls, systems, xd, refs = _batch(cases, 11)
    say("matvec batch, spectra in several rounds", [wl.name + f"/L{wl.pad_L}" for wl in wls])
    ys = matvec_batch([s[0] for s in systems], xd)
    for wl, y, ref in zip(wls, ys, refs):
        assert rel_maxabs(y.cpu().numpy(), ref) < 3e-6, wl.name
