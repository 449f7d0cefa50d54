"""The C ABI of libvoxlod.so without a GPU: the library loads, exports every
function include/voxlod.h declares, and rejects bad arguments on the host
before anything reaches the device."""
import ctypes as C
import os
import re

import pytest

from paper_2110_13368_amd import binding as vb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "voxlod.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vl_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 20
    lib = C.CDLL(vb.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(vb.SIGNATURES)


def test_abi_version():
    assert vb.vl_abi_version() == 1


def _code(fn, *args):
    with pytest.raises(vb.VoxlodError) as e:
        fn(*args)
    return e.value.code


def test_create_rejects_bad_arguments():
    assert _code(vb.vl_create, 0) == vb.VL_E_ARG
    assert _code(vb.vl_create, 1, 7) == vb.VL_E_ARG
    assert _code(vb.vl_create, 1, vb.VL_F32, 9) == vb.VL_E_ARG
    assert "precision" in vb.vl_last_error() or "decay" in vb.vl_last_error()


def test_setup_validation_and_sizes():
    h = vb.vl_create(2, vb.VL_F32)
    try:
        assert _code(vb.vl_set_grid, h, 2, 4, 4, 4, 1, 1, 1, 0, 0, 0) == vb.VL_E_ARG  # sim index
        assert _code(vb.vl_set_grid, h, 0, 0, 4, 4, 1, 1, 1, 0, 0, 0) == vb.VL_E_ARG
        assert _code(vb.vl_set_grid, h, 0, 4, 4, 4, -1, 1, 1, 0, 0, 0) == vb.VL_E_ARG
        assert _code(vb.vl_set_grid, h, 0, 4, 4, 4, 1, float("nan"), 1, 0, 0, 0) == vb.VL_E_ARG
        assert _code(vb.vl_set_grid, h, 0, 1024, 1024, 1024, 1, 1, 1, 0, 0, 0) == vb.VL_E_SHAPE
        assert _code(vb.vl_finalize, h, 0.01) == vb.VL_E_STATE  # no grid yet
        vb.vl_set_grid(h, 0, 50, 40, 30, 20, 20, 20, -500, -400, -300)
        vb.vl_set_grid(h, 1, 7, 1, 3, 10, 10, 10, 0, 0, 0)
        assert _code(vb.vl_set_boundary, h, 0, 0, 0, vb.VL_DIRICHLET, 1.0) == vb.VL_E_ARG  # no substrates
        assert _code(vb.vl_set_substrates, h, 0, [1.0, -2.0], [0.0, 0.0]) == vb.VL_E_ARG
        vb.vl_set_substrates(h, 0, [1e5, 1e3], [0.1, 0.0])
        vb.vl_set_substrates(h, 1, [5e4], [1.0])
        assert _code(vb.vl_set_boundary, h, 0, 0, 6, vb.VL_DIRICHLET, 1.0) == vb.VL_E_ARG
        assert _code(vb.vl_set_boundary, h, 0, 2, 0, vb.VL_DIRICHLET, 1.0) == vb.VL_E_ARG
        assert _code(vb.vl_set_boundary, h, 0, 0, 0, 3, 1.0) == vb.VL_E_ARG
        assert _code(vb.vl_set_boundary, h, 0, 0, 0, vb.VL_DIRICHLET, float("inf")) == vb.VL_E_ARG
        vb.vl_set_boundary(h, 0, 1, 5, vb.VL_DIRICHLET, 38.0)
        assert _code(vb.vl_reserve_cells, h, 0, -1) == vb.VL_E_ARG
        assert _code(vb.vl_reserve_cells, h, 0, (1 << 24) + 1) == vb.VL_E_ARG
        vb.vl_reserve_cells(h, 0, 1000)
        assert _code(vb.vl_resize_cells, h, 0, 10) == vb.VL_E_STATE  # before vl_finalize
        assert _code(vb.vl_finalize, h, 0.0) == vb.VL_E_ARG
        assert _code(vb.vl_step, h, 1) == vb.VL_E_STATE
        assert _code(vb.vl_bind, h, 0, 0, 0) == vb.VL_E_STATE  # not finalized
        fe, wb = vb.vl_finalize(h, 0.01)
        # volumes are padded to 64 floats (256 bytes)
        vol0 = -(-50 * 40 * 30 // 64) * 64
        vol1 = -(-7 * 1 * 3 // 64) * 64
        assert fe == 2 * vol0 + vol1
        assert vb.vl_field_offset(h, 1) == 2 * vol0
        assert vb.vl_volume_stride(h, 0) == vol0
        assert wb > 0 and wb % 256 == 0
        # capacity changed after vl_finalize: the workspace grows and shrinks
        # with it, the field layout does not move
        wb2 = vb.vl_resize_cells(h, 0, 50_000)
        assert wb2 > wb and wb2 % 256 == 0
        assert vb.vl_resize_cells(h, 0, 1000) == wb
        assert _code(vb.vl_resize_cells, h, 0, -1) == vb.VL_E_ARG
        assert _code(vb.vl_resize_cells, h, 0, (1 << 24) + 1) == vb.VL_E_ARG
        assert _code(vb.vl_resize_cells, h, 2, 10) == vb.VL_E_ARG  # no such simulation
        assert vb.vl_field_offset(h, 1) == 2 * vol0
        assert _code(vb.vl_finalize, h, 0.01) == vb.VL_E_STATE
        assert _code(vb.vl_set_grid, h, 0, 4, 4, 4, 1, 1, 1, 0, 0, 0) == vb.VL_E_STATE
        assert _code(vb.vl_bind, h, 0, 0, 0) == vb.VL_E_ARG  # null buffers
        assert _code(vb.vl_bind, h, 256, 4, 0) == vb.VL_E_ARG  # misaligned
        assert _code(vb.vl_step, h, 1) == vb.VL_E_STATE  # not bound
        assert _code(vb.vl_upload_cells, h, 0, [[0, 0, 0]], [1.0], [[1, 1]], [[1, 1]], [[1, 1]], 2) == vb.VL_E_STATE
        assert _code(vb.vl_snapshot, h, 0, 256, 256) == vb.VL_E_STATE  # not bound
        assert _code(vb.vl_snapshot, h, 2, 256, 256) == vb.VL_E_ARG  # no such simulation
        vb.vl_snapshot_wait(h)  # nothing enqueued: returns at once
    finally:
        vb.vl_destroy(h)


def test_fp32_rejects_overlong_lines_fp64_accepts():
    for precision, expect in ((vb.VL_F32, vb.VL_E_SHAPE), (vb.VL_F64, None)):
        h = vb.vl_create(1, precision)
        try:
            vb.vl_set_grid(h, 0, 600, 2, 2, 1, 1, 1, 0, 0, 0)
            vb.vl_set_substrates(h, 0, [1.0], [0.0])
            if expect is None:
                vb.vl_finalize(h, 0.01)
            else:
                assert _code(vb.vl_finalize, h, 0.01) == expect
        finally:
            vb.vl_destroy(h)


def test_options_on_the_host():
    h = vb.vl_create(1, vb.VL_F32)
    try:
        assert vb.vl_get_option(h, vb.VL_OPT_FUSE_SOURCES) == 1
        assert vb.vl_get_option(h, vb.VL_OPT_XCD_ORDER) == 1
        assert vb.vl_get_option(h, vb.VL_OPT_FUSE_XY) == 0
        vb.vl_set_option(h, vb.VL_OPT_FUSE_XY, 1)
        assert vb.vl_get_option(h, vb.VL_OPT_FUSE_XY) == 1
        assert _code(vb.vl_set_option, h, vb.VL_OPT_FUSE_XY, 3) == vb.VL_E_ARG
        assert vb.vl_get_option(h, vb.VL_OPT_X_LANES) == 1
        vb.vl_set_option(h, vb.VL_OPT_X_LANES, 0)
        assert vb.vl_get_option(h, vb.VL_OPT_X_LANES) == 0
        assert _code(vb.vl_set_option, h, vb.VL_OPT_X_LANES, -1) == vb.VL_E_ARG
        assert vb.vl_get_option(h, vb.VL_OPT_ADJOINT_TABLES) == 1
        vb.vl_set_option(h, vb.VL_OPT_ADJOINT_TABLES, 0)
        assert vb.vl_get_option(h, vb.VL_OPT_ADJOINT_TABLES) == 0
        assert _code(vb.vl_set_option, h, vb.VL_OPT_ADJOINT_TABLES, 2) == vb.VL_E_ARG
        assert vb.vl_get_option(h, vb.VL_OPT_Z_SOURCES_STORING) == -1
        vb.vl_set_option(h, vb.VL_OPT_Z_SOURCES_STORING, 1)
        assert vb.vl_get_option(h, vb.VL_OPT_Z_SOURCES_STORING) == 1
        assert _code(vb.vl_set_option, h, vb.VL_OPT_Z_SOURCES_STORING, 2) == vb.VL_E_ARG
        vb.vl_set_option(h, vb.VL_OPT_X_LANES, 2)  # lines of 65 voxels and more
        assert vb.vl_get_option(h, vb.VL_OPT_X_LANES) == 2
        assert _code(vb.vl_set_option, h, vb.VL_OPT_X_LANES, 3) == vb.VL_E_ARG
        assert vb.vl_get_option(h, vb.VL_OPT_X_LANE_LINES) in (1, 2, 4, 8, 16)
        for v in (1, 2, 4, 8, 16):
            vb.vl_set_option(h, vb.VL_OPT_X_LANE_LINES, v)
            assert vb.vl_get_option(h, vb.VL_OPT_X_LANE_LINES) == v
        for v in (0, 3, 32, -4):
            assert _code(vb.vl_set_option, h, vb.VL_OPT_X_LANE_LINES, v) == vb.VL_E_ARG
        vb.vl_set_option(h, vb.VL_OPT_XCD_ORDER, 0)
        assert vb.vl_get_option(h, vb.VL_OPT_XCD_ORDER) == 0
        vb.vl_set_option(h, vb.VL_OPT_FUSE_SOURCES, 2)  # carried into the next x solve
        assert vb.vl_get_option(h, vb.VL_OPT_FUSE_SOURCES) == 2
        assert _code(vb.vl_set_option, h, vb.VL_OPT_FUSE_SOURCES, 3) == vb.VL_E_ARG
        assert _code(vb.vl_set_option, h, vb.VL_OPT_FUSE_SOURCES, -1) == vb.VL_E_ARG
        assert _code(vb.vl_set_option, h, 99, 0) == vb.VL_E_ARG
        # the one-launch step is switched off for now and says so
        assert _code(vb.vl_set_option, h, vb.VL_OPT_STEP_MODE, vb.VL_MODE_PERSISTENT) == vb.VL_E_STATE
        assert "switched off" in vb.vl_last_error()
        assert vb.vl_get_option(h, vb.VL_OPT_STEP_MODE) == vb.VL_MODE_LAUNCHES
    finally:
        vb.vl_destroy(h)
    h = vb.vl_create(1, vb.VL_F64)
    try:
        assert _code(vb.vl_set_option, h, vb.VL_OPT_STEP_MODE, vb.VL_MODE_PERSISTENT) == vb.VL_E_ARG
    finally:
        vb.vl_destroy(h)


def test_destroy_null_is_ok():
    vb.vl_destroy(None)


def test_copy_probe_rejects_bad_arguments_on_the_host():
    # all of these fail before any device call
    assert _code(vb.vl_copy_probe, 0, 256, 1024) == vb.VL_E_ARG  # null destination
    assert _code(vb.vl_copy_probe, 4096, 0, 1024) == vb.VL_E_ARG  # null source
    assert _code(vb.vl_copy_probe, 4096, 8192, 1024, 2) == vb.VL_E_ARG  # width
    assert _code(vb.vl_copy_probe, 4096, 8192, 1024, 16, 5) == vb.VL_E_ARG  # non-temporal bits
    assert _code(vb.vl_copy_probe, 4096, 8192, 1024, 4, 4) == vb.VL_E_ARG  # tiles take width 16
    assert _code(vb.vl_copy_probe, 4096, 8192, 1000) == vb.VL_E_ARG  # not a multiple of 16
    assert _code(vb.vl_copy_probe, 4100, 8192, 1024) == vb.VL_E_ARG  # misaligned
    assert _code(vb.vl_copy_probe, 4096, 4608, 1024) == vb.VL_E_ARG  # overlapping
    assert "overlap" in vb.vl_last_error()
    assert _code(vb.vl_copy_probe, 4096, 4080, 1024) == vb.VL_E_ARG  # overlapping, source above


def test_mass_noalloc_rejects_bad_arguments_on_the_host():
    # all of these fail before any device call
    assert _code(vb.vl_mass_noalloc, 0, vb.VL_F32, 10, 1, 10, 4096) == vb.VL_E_ARG  # null field
    assert _code(vb.vl_mass_noalloc, 4096, vb.VL_F32, 10, 1, 10, 0) == vb.VL_E_ARG  # null output
    assert _code(vb.vl_mass_noalloc, 4096, 5, 10, 1, 10, 4096) == vb.VL_E_ARG  # precision
    assert _code(vb.vl_mass_noalloc, 4096, vb.VL_F32, 0, 1, 10, 4096) == vb.VL_E_ARG  # no voxels
    assert _code(vb.vl_mass_noalloc, 4096, vb.VL_F32, 10, 0, 10, 4096) == vb.VL_E_ARG  # no volumes
    assert _code(vb.vl_mass_noalloc, 4096, vb.VL_F32, 10, 65, 10, 4096) == vb.VL_E_SHAPE  # past the array
    assert "64 volumes" in vb.vl_last_error()
    assert _code(vb.vl_mass_noalloc, 4096, vb.VL_F32, 10, 2, 9, 4096) == vb.VL_E_ARG  # overlapping volumes
    assert _code(vb.vl_mass_noalloc, 4098, vb.VL_F32, 10, 1, 10, 4096) == vb.VL_E_ARG  # misaligned field
    assert _code(vb.vl_mass_noalloc, 4096, vb.VL_F64, 10, 1, 10, 4100) == vb.VL_E_ARG  # misaligned output


def _roctx():
    """The roctx library that libvoxlod.so loaded (its path from this process's maps)."""
    C.CDLL(vb.LIB_PATH)
    paths = {ln.split()[-1] for ln in open("/proc/self/maps") if "librocprofiler-sdk-roctx" in ln}
    assert len(paths) == 1, paths
    r = C.CDLL(paths.pop())
    r.roctxRangePushA.restype, r.roctxRangePushA.argtypes = C.c_int, [C.c_char_p]
    r.roctxRangePop.restype = C.c_int
    return r


def test_calls_close_the_roctx_ranges_they_open():
    # every entry point that opens a range (rocprofv3 --marker-trace) closes it
    # on each return path, including the early error returns
    r = _roctx()
    assert r.roctxRangePushA(b"probe") == 0 and r.roctxRangePop() == 0
    h = vb.vl_create(1, vb.VL_F32)
    try:
        assert _code(vb.vl_finalize, h, 0.01) == vb.VL_E_STATE  # no grid: returns inside its range
        assert _code(vb.vl_step, h, 1) == vb.VL_E_STATE  # not bound
        assert _code(vb.vl_tune, h, None) == vb.VL_E_STATE
        assert _code(vb.vl_resize_cells, h, 0, 10) == vb.VL_E_STATE
        vb.vl_set_grid(h, 0, 9, 8, 7, 10, 10, 10, 0, 0, 0)
        vb.vl_set_substrates(h, 0, [1e3], [0.1])
        vb.vl_finalize(h, 0.01)
        assert _code(vb.vl_step, h, 1) == vb.VL_E_STATE  # finalized, not bound
    finally:
        vb.vl_destroy(h)
    # nothing is left open on this thread: a new range starts at level 0
    assert r.roctxRangePushA(b"probe") == 0
    assert r.roctxRangePop() == 0
