"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes workspaces on the host, and rejects bad arguments
before launching anything."""
import ctypes
import os
import re

import pytest

from paper_2509_03015_amd import _binding as bb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "bds.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(bds_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bb.LIB_PATH):
        from paper_2509_03015_amd import build
        build.build()
    return bb.load()


def test_header_declares_the_entry_points():
    fns = header_functions()
    for f in ("bds_factor", "bds_solve", "bds_factor_batched", "bds_solve_batched", "bds_backward",
              "bds_workspace_size", "bds_batched_workspace_size"):
        assert f in fns
    assert set(fns) == set(bb.EXPORTS)


def test_library_exports_every_header_symbol(lib):
    for f in header_functions():
        assert hasattr(lib, f), f
    assert b"gfx950" in lib.bds_version()


def desc(N=64, n=16, d=1, prec=0, nstar=0, max_refine=0, tiles=0, tol=0.0):
    return bb.BdsDesc(N, n, d, prec, nstar, max_refine, tiles, tol)


def test_workspace_sizes_follow_the_level_plan(lib):
    rc, f, s = bb.workspace_size(desc(64, 16, 1))
    assert rc == 0
    # levels M = 64, 32, 16, 8, 4, 2 (nstar = 1): interiors 32+16+8+4+2+1 = 63
    blk = 16 * 16 * 8
    interiors = 63
    nxt_d = 32 + 16 + 8 + 4 + 2 + 1
    nxt_s = 31 + 15 + 7 + 3 + 1 + 0
    lower = (3 * interiors + nxt_d + nxt_s) * blk + (1 + 0 + 1) * blk
    assert lower <= f <= lower + 256 * 40
    rc2, f2, s2 = bb.workspace_size(desc(64, 16, 7))
    assert rc2 == 0 and f2 == f and s2 > s
    rc3, f3, _ = bb.workspace_size(desc(64, 16, 1, prec=1))
    assert rc3 == 0 and f3 < f            # FP32 levels, FP64 coarse
    rc4, f4, _ = bb.workspace_size(desc(64, 16, 1, nstar=64))
    assert rc4 == 0 and f4 < f            # no reduction level at all


def test_padding_to_multiple_of_16(lib):
    _, f17, _ = bb.workspace_size(desc(10, 17, 1))
    _, f32, _ = bb.workspace_size(desc(10, 32, 1))
    assert f17 > f32                      # same padded blocks plus the padded input copies


@pytest.mark.parametrize("bad", [dict(N=0), dict(n=0), dict(n=257), dict(d=0), dict(prec=7), dict(nstar=-1),
                                 dict(max_refine=-2), dict(tol=-1.0), dict(tiles=5), dict(tiles=1 << 12),
                                 dict(tiles=bb.tiles(solve=bb.BDS_TILE_G64), n=64),
                                 dict(tiles=bb.tiles(couple=bb.BDS_TILE_W32), n=16),
                                 dict(tiles=bb.tiles(schur=bb.BDS_TILE_G64), n=32),
                                 dict(tiles=bb.tiles(couple=bb.BDS_TILE_G128), n=64)])
def test_invalid_descriptors_rejected(lib, bad):
    kw = dict(N=8, n=4, d=1)
    kw.update(bad)
    rc, _, _ = bb.workspace_size(desc(**kw))
    assert rc == bb.BDS_EINVAL


def test_calls_reject_bad_arguments_without_launching(lib):
    d = desc(8, 4, 1)
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.bds_factor(ctypes.byref(d), null, null, fake, 1 << 20, fake, null) == bb.BDS_EINVAL
    assert lib.bds_factor(ctypes.byref(d), fake, fake, fake, 16, fake, null) == bb.BDS_EWORKSPACE
    assert lib.bds_solve(ctypes.byref(d), fake, 1 << 30, null, null, fake, fake, fake, 1 << 30, fake,
                         null) == bb.BDS_EINVAL  # B == X
    assert lib.bds_solve(ctypes.byref(d), fake, 16, null, null, fake, ctypes.c_void_p(0x2000), fake, 1 << 30,
                         fake, null) == bb.BDS_EWORKSPACE
    mixed = desc(8, 4, 1, prec=1)
    assert lib.bds_solve(ctypes.byref(mixed), fake, 1 << 30, null, null, fake, ctypes.c_void_p(0x2000), fake,
                         1 << 30, fake, null) == bb.BDS_EINVAL  # refinement needs A
    assert lib.bds_backward(ctypes.byref(d), fake, 1 << 30, null, null, fake, fake, null, fake, fake, fake,
                            1 << 30, fake, null) == bb.BDS_EINVAL
    bad = desc(0, 4, 1)
    assert lib.bds_factor(ctypes.byref(bad), fake, fake, fake, 1 << 20, fake, null) == bb.BDS_EINVAL


def descs_array(specs, prec=0, nstar=0):
    arr = (bb.BdsDesc * len(specs))()
    for k, (N, n, d) in enumerate(specs):
        arr[k] = bb.BdsDesc(N, n, d, prec, nstar, 0, 0, 0.0)
    return arr


def test_batched_workspace_is_sum_of_systems_plus_tables(lib):
    specs = [(10, 8, 1), (100, 32, 4), (1, 3, 2)]
    arr = descs_array(specs)
    f = ctypes.c_size_t(0)
    s = ctypes.c_size_t(0)
    assert lib.bds_batched_workspace_size(3, arr, ctypes.byref(f), ctypes.byref(s)) == 0
    single = [bb.workspace_size(desc(N, n, d)) for N, n, d in specs]
    assert f.value > sum(x[1] for x in single)
    assert s.value > sum(x[2] for x in single)


def test_batched_rejects_mixed_precision_and_bad_members(lib):
    f = ctypes.c_size_t(0)
    s = ctypes.c_size_t(0)
    arr = descs_array([(10, 8, 1), (20, 16, 1)])
    arr[1].prec = 1
    assert lib.bds_batched_workspace_size(2, arr, ctypes.byref(f), ctypes.byref(s)) == bb.BDS_EINVAL
    arr = descs_array([(10, 8, 1), (0, 16, 1)])
    assert lib.bds_batched_workspace_size(2, arr, ctypes.byref(f), ctypes.byref(s)) == bb.BDS_EINVAL
    assert lib.bds_batched_workspace_size(0, arr, ctypes.byref(f), ctypes.byref(s)) == bb.BDS_EINVAL
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    good = descs_array([(10, 8, 1), (20, 16, 1)])
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0)  # second Ad missing
    assert lib.bds_factor_batched(2, good, ptrs, ptrs, fake, 1 << 30, fake, null) == bb.BDS_EINVAL
    ok = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    assert lib.bds_factor_batched(2, good, ok, ok, fake, 16, fake, null) == bb.BDS_EWORKSPACE
    same = (ctypes.c_void_p * 2)(0x3000, 0x4000)
    assert lib.bds_solve_batched(2, good, fake, 1 << 30, null, null, same, same, fake, 1 << 30, fake,
                                 null) == bb.BDS_EINVAL  # B[k] == X[k]


def test_trace_enable_bounds(lib):
    assert lib.bds_trace_enable(-1) == bb.BDS_EINVAL
    assert lib.bds_trace_enable(1 << 21) == bb.BDS_EINVAL
    assert lib.bds_trace_enable(0) == bb.BDS_OK


@pytest.mark.parametrize("n,t", [(16, bb.tiles(bb.BDS_TILE_W16, bb.BDS_TILE_W16, bb.BDS_TILE_W16)),
                                 (32, bb.tiles(bb.BDS_TILE_W32, bb.BDS_TILE_W16, bb.BDS_TILE_W32)),
                                 (64, bb.tiles(bb.BDS_TILE_G64, bb.BDS_TILE_W32, bb.BDS_TILE_W16)),
                                 (128, bb.tiles(bb.BDS_TILE_G128, bb.BDS_TILE_G64, bb.BDS_TILE_W32)),
                                 (256, bb.tiles(schur=bb.BDS_TILE_G128))])
def test_tile_choices_that_fit_are_accepted_and_do_not_change_workspaces(lib, n, t):
    rc, f, s = bb.workspace_size(desc(40, n, 3, tiles=t))
    rc0, f0, s0 = bb.workspace_size(desc(40, n, 3))
    assert rc == 0 and rc0 == 0 and (f, s) == (f0, s0)


def test_tune_workspace_covers_every_nstar_candidate(lib):
    rc, f, s = bb.tune_workspace_size(desc(100, 32, 2))
    assert rc == 0
    for ns in (1, 2, 4, 8, 16, 32, 64):
        rc1, f1, s1 = bb.workspace_size(desc(100, 32, 2, nstar=ns))
        assert rc1 == 0 and f1 <= f and s1 <= s
    # a fixed nstar is not searched
    assert bb.tune_workspace_size(desc(100, 32, 2, nstar=8))[1:] == bb.workspace_size(desc(100, 32, 2, nstar=8))[1:]
    assert bb.tune_workspace_size(desc(0, 32, 2))[0] == bb.BDS_EINVAL


def test_tune_rejects_bad_arguments_without_launching(lib):
    d = desc(8, 4, 1)
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    best = bb.BdsDesc()
    assert lib.bds_tune(ctypes.byref(d), fake, fake, fake, fake, fake, 1 << 30, fake, 1 << 30, fake, 3, null,
                        None) == bb.BDS_EINVAL          # no output descriptor
    assert lib.bds_tune(ctypes.byref(d), fake, fake, fake, fake, fake, 16, fake, 1 << 30, fake, 3, null,
                        ctypes.byref(best)) == bb.BDS_EWORKSPACE
    bad = desc(8, 4, 1, tiles=9)
    assert lib.bds_tune(ctypes.byref(bad), fake, fake, fake, fake, fake, 1 << 30, fake, 1 << 30, fake, 3, null,
                        ctypes.byref(best)) == bb.BDS_EINVAL
