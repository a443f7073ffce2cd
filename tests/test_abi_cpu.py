"""CPU checks of the C ABI: the library loads, exports every function that
include/tt.h declares, and rejects bad arguments before touching a device."""
import ctypes as C

import numpy as np
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tt.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1806_07938_amd import tt
    return tt.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "tt_solve_frame" in names and "tt_matvec" in names
    for name in names:
        assert hasattr(lib, name), name
    from paper_1806_07938_amd import tt
    assert sorted(tt.EXPORTED) == names


def test_status_strings(lib):
    for code, name in enumerate(["TT_OK", "TT_INVALID_ARG", "TT_HIP_ERROR", "TT_OUT_OF_MEMORY",
                                 "TT_NOT_CONVERGED", "TT_BREAKDOWN", "TT_NOT_READY"]):
        assert lib.tt_status_string(code).decode() == name
    assert lib.tt_status_string(99).decode() == "TT_UNKNOWN_STATUS"


def test_null_arguments_rejected(lib):
    from paper_1806_07938_amd import tt
    assert lib.tt_create(None, 0, None) == tt.TT_INVALID_ARG
    out = C.c_void_p()
    assert lib.tt_generate_kernels(None, None, None, C.byref(out)) == tt.TT_INVALID_ARG
    assert "NULL" in lib.tt_last_error().decode()
    assert lib.tt_matvec(None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_matvec_noalloc(None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_learned_create(None, 0, 6, 32, 0) == tt.TT_INVALID_ARG
    assert lib.tt_learned_destroy(None) == tt.TT_OK
    assert lib.tt_learned_apply(None, None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_learned_train_step(None, None, None, None, 1, 1e-3, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_learned_train(None, None, 1, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_set_learned(None, None) == tt.TT_INVALID_ARG
    assert lib.tt_learned_weight_count(None, None) == tt.TT_INVALID_ARG
    assert lib.tt_solve_frame(None, None, None, None, None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_project(None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_kernels_copy(None, None, 0) == tt.TT_INVALID_ARG
    assert lib.tt_destroy(None) == tt.TT_OK
    assert lib.tt_kernels_destroy(None) == tt.TT_OK
    # batched product: an empty batch is a no-op, missing arrays and negative counts are refused
    assert lib.tt_matvec_batch(None, 0, None, None, None) == tt.TT_OK
    assert lib.tt_matvec_batch(None, 1, None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_matvec_batch(None, -1, None, None, None) == tt.TT_INVALID_ARG
    assert lib.tt_solve_batch(None, 0, None, None, None, None, None, None) == tt.TT_OK
    assert lib.tt_solve_batch(None, 2, None, None, None, None, None, None) == tt.TT_INVALID_ARG


def test_batch_workload_family():
    # distinct 74x74 systems for the batched product: same geometry, seeded
    # weights (normalised, decaying with altitude on average) and r0 in range
    import workloads as W
    base = W.lgs6_74x74(pad_L=256)
    fam = [W.lgs6_74x74_family(i) for i in range(4)]
    assert W.lgs6_74x74_family(-1).name == "lgs6_74x74"
    for wl in fam:
        assert wl.pad_L == 256 and wl.n == 74 and wl.n_vs == 3972 and wl.n_gs == 6
        assert np.array_equal(wl.valid, base.valid) and np.allclose(wl.h, base.h)
        assert abs(wl.w.sum() - 1.0) < 1e-12 and (wl.w > 0).all()
        assert 0.10 <= wl.r0 <= 0.25
    assert len({round(wl.r0, 12) for wl in fam}) == 4
    assert all(not np.allclose(fam[0].w, wl.w) for wl in fam[1:])
    again = W.lgs6_74x74_family(2)
    assert again.r0 == fam[2].r0 and np.array_equal(again.w, fam[2].w)


def test_struct_layouts_match_header():
    # field order and sizes of the ctypes mirrors agree with the C structs
    from paper_1806_07938_amd import tt
    text = open(HEADER).read()
    for cname, py in (("tt_geometry", tt._Geometry), ("tt_atmosphere", tt._Atmosphere),
                      ("tt_target", tt._Target), ("tt_solve_opts", tt._SolveOpts),
                      ("tt_solve_info", tt._SolveInfo), ("tt_system_info", tt._SystemInfo),
                      ("tt_train_opts", tt._TrainOpts), ("tt_train_info", tt._TrainInfo)):
        body = re.search(r"typedef struct \{((?:(?!typedef).)*?)\}\s*" + cname + ";", text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = re.sub(r"\b(const|unsigned|char|int|double|size_t)\b|\*", " ", decl).strip()
            fields += [nm.strip() for nm in decl.split(",") if nm.strip()]
        assert [f for f, _ in py._fields_] == fields, cname


def test_no_device_reports_error_not_crash(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1806_07938_amd import tt
    h = C.c_void_p()
    st = lib.tt_create(C.byref(h), 0, None)
    assert st in (tt.TT_HIP_ERROR, tt.TT_INVALID_ARG)
    assert lib.tt_last_error().decode() != ""


@pytest.mark.parametrize("n,D,obs,count", [(10, 8.0, 0.30, 76), (74, 39.0, 0.28, 3972),
                                           (40, 0.52703 * 40, 0.28, 1168), (60, 0.52703 * 60, 0.28, 2612),
                                           (84, 0.52703 * 84, 0.28, 5112)])
def test_library_pupil_rule_matches_workloads(lib, n, D, obs, count):
    """tt_pupil_mask (host only, exact areas) against the seeded workloads' mask
    (the same half-area rule measured on a 64 x 64 point grid per subaperture)."""
    import workloads as W
    from paper_1806_07938_amd import tt
    m = tt.pupil_mask(n, D, obs)
    assert int(m.sum()) == count
    assert np.array_equal(m, W.pupil_mask(n, D, obs))


def test_library_pupil_rule_limits(lib):
    from paper_1806_07938_amd import tt
    assert tt.pupil_mask(4, 2.0, 0.0).sum() == 12        # a disk inscribed in 4 x 4 squares: the corners go
    assert tt.pupil_mask(1, 1.0, 0.0).all()               # pi/4 of one square
    assert not tt.pupil_mask(2, 2.0, 0.9).any()           # a thin annulus covers < 1/2 of every square
    out = (C.c_ubyte * 16)()
    assert lib.tt_pupil_mask(4, 1.0, 1.0, out, None) == tt.TT_INVALID_ARG
    assert lib.tt_pupil_mask(0, 1.0, 0.0, out, None) == tt.TT_INVALID_ARG
    assert lib.tt_pupil_mask(4, -1.0, 0.0, out, None) == tt.TT_INVALID_ARG
    assert lib.tt_pupil_mask(4, 1.0, 0.0, None, None) == tt.TT_INVALID_ARG
