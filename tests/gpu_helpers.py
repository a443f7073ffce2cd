"""Helpers shared by the GPU parity tests: build a library system from a
seeded workload and the matching oracle objects."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def make_system(wl, target=True, pad_L=None, proj_pad_L=0, n_prime=0):
    from paper_1806_07938_amd import Context, system_from
    ctx = Context(0)
    k = system_from(ctx, wl, target=target, pad_L=pad_L, proj_pad_L=proj_pad_L, n_prime=n_prime)
    return ctx, k


def oracle_tables_packed(wl):
    """Oracle tables in the library's copy layout [pair(g<=h)][xx, xy, yy][v][u]."""
    from oracle.covariance import kernel_table
    out = []
    for g in range(wl.n_gs):
        for h in range(g, wl.n_gs):
            out.append([kernel_table(wl, g, h, 0, 0), kernel_table(wl, g, h, 0, 1), kernel_table(wl, g, h, 1, 1)])
    return np.array(out)


def rel_maxabs(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
