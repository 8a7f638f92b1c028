"""The C ABI library builds, loads and exports every declared symbol; host-only
argument checks (no device work, no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpals.h")


def _lib():
    from paper_2010_12056_amd import build_lib, cpals

    if not os.path.exists(cpals.LIB_PATH):
        build_lib.build()
    return cpals.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("cp_mttkrp", "cp_als_sweep", "cp_pp_sweep", "cp_plan_create", "cp_set_tensor"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    # and the binding declares a signature for each of them
    from paper_2010_12056_amd import cpals

    assert set(_declared()) == set(cpals.EXPORTS)


def test_status_strings():
    L = _lib()
    for s in range(7):
        assert L.cp_status_str(s)
    assert L.cp_status_str(99) == b"unknown status"


def test_plan_create_argument_checks():
    from paper_2010_12056_amd import cpals

    L = _lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 4)(8, 8, 8, 8)
    assert L.cp_plan_create(ctypes.byref(h), 2, dims, 4, cpals.CP_F32, cpals.CP_TREE_DT, None) == cpals.CP_ERR_UNSUPPORTED
    assert L.cp_plan_create(ctypes.byref(h), 4, dims, 0, cpals.CP_F32, cpals.CP_TREE_DT, None) == cpals.CP_ERR_UNSUPPORTED
    assert L.cp_plan_create(ctypes.byref(h), 4, dims, 129, cpals.CP_F32, cpals.CP_TREE_DT, None) == cpals.CP_ERR_UNSUPPORTED
    assert L.cp_plan_create(ctypes.byref(h), 4, dims, 4, 8, cpals.CP_TREE_DT, None) == cpals.CP_ERR_UNSUPPORTED
    bad = (ctypes.c_int64 * 4)(8, 0, 8, 8)
    assert L.cp_plan_create(ctypes.byref(h), 4, bad, 4, cpals.CP_F32, cpals.CP_TREE_DT, None) == cpals.CP_ERR_ARG
    assert L.cp_plan_create(None, 4, dims, 4, cpals.CP_F32, cpals.CP_TREE_DT, None) == cpals.CP_ERR_ARG
    assert L.cp_plan_create(ctypes.byref(h), 4, dims, 4, cpals.CP_F32, 3, None) == cpals.CP_ERR_UNSUPPORTED


def test_combined_tree_accepted_at_every_order():
    """CP_TREE_DT_COMBINED is a valid tree at orders 3 (where it is the
    standard tree) and up; the workspace also holds the Khatri-Rao operand of
    the last two modes (s_{N-2} s_{N-1} x R)."""
    from paper_2010_12056_amd import cpals

    L = _lib()
    for dims_t in ((40, 30, 20), (256, 256, 33, 3), (12, 10, 9, 8, 7)):
        dims = (ctypes.c_int64 * len(dims_t))(*dims_t)
        sizes = {}
        for tree in (cpals.CP_TREE_DT, cpals.CP_TREE_DT_COMBINED):
            h = ctypes.c_void_p()
            assert L.cp_plan_create(ctypes.byref(h), len(dims_t), dims, 50, cpals.CP_F32, tree, None) == cpals.CP_OK
            n = ctypes.c_size_t()
            assert L.cp_plan_workspace_size(h, ctypes.byref(n)) == cpals.CP_OK
            sizes[tree] = n.value
            assert L.cp_plan_destroy(h) == cpals.CP_OK
        krp = dims_t[-2] * dims_t[-1] * 50 * 4 if len(dims_t) >= 4 else 0
        assert sizes[cpals.CP_TREE_DT_COMBINED] >= sizes[cpals.CP_TREE_DT] + krp - 256  # regions are 256-aligned


def test_profile_mask_checked():
    from paper_2010_12056_amd import cpals

    L = _lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    assert L.cp_plan_create(ctypes.byref(h), 3, dims, 4, cpals.CP_F32, cpals.CP_TREE_DT, None) == cpals.CP_OK
    for mask in (0, 1, 0b10101, 31):
        assert L.cp_profile_enable(h, mask) == cpals.CP_OK
    for mask in (-1, 32, 1 << 20):
        assert L.cp_profile_enable(h, mask) == cpals.CP_ERR_ARG
    assert L.cp_plan_destroy(h) == cpals.CP_OK


def test_workspace_size_and_state_errors():
    from paper_2010_12056_amd import cpals

    L = _lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 4)(128, 128, 128, 128)
    assert L.cp_plan_create(ctypes.byref(h), 4, dims, 64, cpals.CP_F32, cpals.CP_TREE_MSDT, None) == cpals.CP_OK
    n = ctypes.c_size_t()
    assert L.cp_plan_workspace_size(h, ctypes.byref(n)) == cpals.CP_OK
    # one first-level node (128^3 x 64 FP32 = 512 MiB) dominates
    assert 512 * 2**20 < n.value < 600 * 2**20
    # no workspace, no tensor: sweeps refuse before touching the device
    A = (ctypes.c_void_p * 4)()
    assert L.cp_als_sweep(h, A, None) == cpals.CP_ERR_STATE
    assert b"workspace" in L.cp_last_error(h)
    assert L.cp_plan_set_workspace(h, ctypes.c_void_p(256), 16) == cpals.CP_ERR_ARG
    assert L.cp_plan_destroy(h) == cpals.CP_OK


def test_batch_create_layout_and_argument_checks():
    """Batched path, host side: limits (1 <= s <= 96, 1 <= R <= 32), the
    packed layout (tensors 16-byte aligned, factors back to back, offsets by
    the caller's order) and the launch / workspace argument checks."""
    from paper_2010_12056_amd import cpals

    L = _lib()
    L.cp_batch_destroy.restype = None
    b = ctypes.c_void_p()

    def dims_of(lst):
        return (ctypes.c_int64 * (3 * len(lst)))(*[x for d in lst for x in d])

    def ranks_of(lst):
        return (ctypes.c_int * len(lst))(*lst)

    assert L.cp_batch_create(ctypes.byref(b), 0, dims_of([(4, 4, 4)]), ranks_of([2]), None) == cpals.CP_ERR_ARG
    assert L.cp_batch_create(None, 1, dims_of([(4, 4, 4)]), ranks_of([2]), None) == cpals.CP_ERR_ARG
    for bad_dims, bad_r in (((97, 4, 4), 2), ((4, 0, 4), 2), ((4, 4, 4), 33), ((4, 4, 4), 0)):
        assert L.cp_batch_create(ctypes.byref(b), 1, dims_of([bad_dims]), ranks_of([bad_r]), None) == \
            cpals.CP_ERR_UNSUPPORTED
    shapes = [(3, 5, 7), (16, 16, 16), (1, 1, 1), (96, 2, 9)]
    ranks = [3, 32, 1, 8]
    assert L.cp_batch_create(ctypes.byref(b), 4, dims_of(shapes), ranks_of(ranks), None) == cpals.CP_OK
    toff = (ctypes.c_int64 * 4)()
    aoff = (ctypes.c_int64 * 12)()
    ttot, atot = ctypes.c_int64(), ctypes.c_int64()
    assert L.cp_batch_layout(b, toff, aoff, ctypes.byref(ttot), ctypes.byref(atot)) == cpals.CP_OK
    padded = [-(-(x * y * z) // 4) * 4 for x, y, z in shapes]
    assert ttot.value == sum(padded)
    assert atot.value == sum(sum(d) * r for d, r in zip(shapes, ranks))
    # tensors: disjoint, 16-byte aligned, covering [0, t_total)
    spans = sorted((toff[i], padded[i]) for i in range(4))
    assert all(o % 4 == 0 for o, _ in spans)
    assert spans[0][0] == 0 and all(spans[i][0] + spans[i][1] == spans[i + 1][0] for i in range(3))
    # factors: each of s_m x R, disjoint, covering [0, a_total)
    fac = sorted((aoff[3 * i + m], shapes[i][m] * ranks[i]) for i in range(4) for m in range(3))
    assert fac[0][0] == 0 and all(fac[j][0] + fac[j][1] == fac[j + 1][0] for j in range(11))
    assert L.cp_batch_set_launch(b, 3, 1) == cpals.CP_ERR_UNSUPPORTED
    assert L.cp_batch_set_launch(b, 8, 0) == cpals.CP_ERR_UNSUPPORTED
    assert L.cp_batch_set_launch(b, 8, 1) == cpals.CP_OK
    n = ctypes.c_size_t()
    assert L.cp_batch_workspace_size(b, ctypes.byref(n)) == cpals.CP_OK and n.value > 0
    assert L.cp_batch_set_workspace(b, ctypes.c_void_p(256 + 8), n.value) == cpals.CP_ERR_ARG  # misaligned
    assert L.cp_batch_set_workspace(b, ctypes.c_void_p(256), n.value - 1) == cpals.CP_ERR_ARG  # too small
    L.cp_batch_destroy(b)


def test_low_precision_plans_share_the_factor_staging():
    """BF16 and FP8 tensors use the same BF16 factor staging: equal workspace
    per factor variant, the split variants one more transposed factor; the
    E4M3 factor of FP8 x FP8 fits in the same space."""
    from paper_2010_12056_amd import cpals

    L = _lib()
    dims = (ctypes.c_int64 * 3)(96, 80, 72)
    need = {}
    for prec in (cpals.CP_F32, cpals.CP_BF16, cpals.CP_BF16X2, cpals.CP_FP8, cpals.CP_FP8X2, cpals.CP_FP8F8):
        h = ctypes.c_void_p()
        assert L.cp_plan_create(ctypes.byref(h), 3, dims, 40, prec, cpals.CP_TREE_DT, None) == cpals.CP_OK
        n = ctypes.c_size_t()
        assert L.cp_plan_workspace_size(h, ctypes.byref(n)) == cpals.CP_OK
        need[prec] = n.value
        assert L.cp_plan_destroy(h) == cpals.CP_OK
    assert need[cpals.CP_FP8] == need[cpals.CP_BF16] and need[cpals.CP_FP8X2] == need[cpals.CP_BF16X2]
    # FP8 x FP8: the E4M3 factor and its column scales fit the BF16 factor's space
    assert need[cpals.CP_FP8F8] == need[cpals.CP_FP8]
    pitch = (96 + 63) // 64 * 64  # the longest mode, padded to the 64-index chunk
    assert need[cpals.CP_BF16X2] - need[cpals.CP_BF16] >= 40 * pitch * 2 - 256  # regions 256-byte aligned
    assert need[cpals.CP_BF16] > need[cpals.CP_F32]
    # the FP32 tensor with three-part BF16 products: its three factor parts
    h = ctypes.c_void_p()
    assert L.cp_plan_create(ctypes.byref(h), 3, dims, 40, cpals.CP_F32X3, cpals.CP_TREE_DT, None) == cpals.CP_OK
    n = ctypes.c_size_t()
    assert L.cp_plan_workspace_size(h, ctypes.byref(n)) == cpals.CP_OK
    assert n.value - need[cpals.CP_F32] >= 3 * 40 * pitch * 2 - 256
    assert L.cp_plan_destroy(h) == cpals.CP_OK
    assert L.cp_plan_create(ctypes.byref(h), 3, dims, 40, 8, cpals.CP_TREE_DT, None) == cpals.CP_ERR_UNSUPPORTED


def test_static_mttkrp_argument_checks():
    """The allocation-free MTTKRP checks its arguments and the size of its
    intermediates against the static scratch before touching the device."""
    from paper_2010_12056_amd import cpals

    L = _lib()
    dims = (ctypes.c_int64 * 4)(16, 16, 16, 16)
    A = (ctypes.c_void_p * 4)(256, 256, 256, 256)
    T = ctypes.c_void_p(256)
    M = ctypes.c_void_p(256)
    f = L.cp_mttkrp_static
    assert f(4, dims, 8, cpals.CP_F32, None, A, 0, M, None) == cpals.CP_ERR_ARG
    assert f(4, dims, 8, cpals.CP_F32, T, A, 4, M, None) == cpals.CP_ERR_ARG
    assert f(2, dims, 8, cpals.CP_F32, T, A, 0, M, None) == cpals.CP_ERR_UNSUPPORTED
    assert f(4, dims, 129, cpals.CP_F32, T, A, 0, M, None) == cpals.CP_ERR_UNSUPPORTED
    A[2] = None
    assert f(4, dims, 8, cpals.CP_F32, T, A, 0, M, None) == cpals.CP_ERR_ARG
    assert b"null factor 2" in L.cp_last_error(None)
    A[2] = 256
    big = (ctypes.c_int64 * 4)(128, 128, 128, 128)  # first node 128^3 x 64 FP32 = 512 MiB
    assert f(4, big, 64, cpals.CP_F32, T, A, 0, M, None) == cpals.CP_ERR_UNSUPPORTED
    assert b"static scratch" in L.cp_last_error(None)
