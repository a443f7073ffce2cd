"""GPU test of tt_matvec_noalloc, the product for callers that cannot
allocate: through the C ABI it must give tt_matvec's result (same kernels:
bitwise equal), on two calls in a row with the second on a smaller system,
with mode removal (its projected input also lives in the fixed array), and
it must refuse a system whose work buffers exceed the array."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_system, say, torch_dev
from oracle.toeplitz import ToeplitzOperator

pytestmark = pytest.mark.gpu


def _x(n, seed):
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)


def _check_pair(ctx, x_host, label):
    import torch
    dev = torch_dev()
    x = torch.tensor(x_host, device=dev)
    y_ref = ctx.matvec(x)
    y_na = torch.full_like(y_ref, float("nan"))
    ctx.matvec_noalloc(x, y_na)
    torch.cuda.synchronize()
    a, b = y_na.cpu().numpy(), y_ref.cpu().numpy()
    say(f"{label}: n_slopes={a.size} max|noalloc - matvec|={np.abs(a - b).max():.3e}")
    assert np.array_equal(a, b), label
    return a


def test_noalloc_matches_matvec_twice_smaller_second():
    big = W.lgs6_74x74()
    small = W.lgs3_10x10()
    ctx_b, kb = make_system(big, target=False)
    ctx_s, ks = make_system(small, target=False)
    # first call: the 74x74 system (1.07 MB of work buffers)
    xb = _x(ctx_b.info["n_slopes"], 1)
    yb = _check_pair(ctx_b, xb, "74x74 L=148")
    # second call: a smaller system; the array keeps the first call's contents
    xs = _x(ctx_s.info["n_slopes"], 2)
    ys = _check_pair(ctx_s, xs, "10x10 L=20")
    # the small product against the oracle's FP64 2RBT product at the FP32 bar
    ref = ToeplitzOperator(small)(xs.astype(np.float64))
    err = np.abs(ys - ref).max() / np.abs(ref).max()
    say(f"10x10: rel max-abs error vs the oracle {err:.2e}")
    assert err < 1e-5
    assert np.isfinite(yb).all()
    # the first system again after the smaller one
    _check_pair(ctx_b, _x(ctx_b.info["n_slopes"], 3), "74x74 again")
    for o in (ctx_b, ctx_s, kb, ks):
        o.close()


def test_noalloc_with_mode_removal():
    wl = W.lgs3_10x10()
    ctx, k = make_system(wl, target=False)
    ctx.set_mode_removal(True)
    _check_pair(ctx, _x(ctx.info["n_slopes"], 4), "10x10 with mode removal")
    ctx.close()
    k.close()


def test_noalloc_refuses_systems_beyond_the_array():
    import torch
    from paper_1806_07938_amd import Context
    from paper_1806_07938_amd.tt import TTError, TT_INVALID_ARG
    n, L = 400, 800      # 2 (L/2 + 1) 4 n complex floats = 10.3 MB > 8 MiB
    ctx = Context(0)
    valid = np.ones((n, n), dtype=np.uint8)
    k = ctx.generate_kernels(n, 2, L, 40.0, np.inf, [[0.0, 0.0], [1e-4, 0.0]], valid, [0.0], [1.0], 0.15, 25.0)
    ctx.set_system(k, noise_scalar=0.1)
    m = ctx.info["n_slopes"]
    x = torch.zeros(m, dtype=torch.float32, device=torch_dev())
    y = torch.zeros_like(x)
    with pytest.raises(TTError) as e:
        ctx.matvec_noalloc(x, y)
    say(str(e.value))
    assert e.value.status == TT_INVALID_ARG and "scratch" in str(e.value)
    ctx.close()
    k.close()
