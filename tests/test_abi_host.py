"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2602_23040_amd import _abi as abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "packuv_gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    fns = header_functions()
    for name in ("pg_atlas_fetch", "pg_project", "pg_bin_sort", "pg_render_fwd", "pg_render_bwd", "pg_project_bwd"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    lib = abi.lib()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(abi.SIGNATURES), "binding and header disagree"


def _cam(**kw):
    import numpy as np
    import synth
    c = synth.pinhole(np.eye(3), np.zeros(3), 64, 48)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,needle", [
    (dict(fx=0.0), "fx and fy"),
    (dict(width=0), "width and height"),
    (dict(frame=3), "frame out of range"),
])
def test_views_create_rejects_bad_cameras(kw, needle):
    with pytest.raises(abi.PGError) as e:
        abi.pg_views_create([_cam(**kw)], 1, 10, 0, abi.make_tiling())
    assert e.value.status == -1 and needle in str(e.value)


@pytest.mark.parametrize("tiling", [(16, 8, 256), (8, 32, 100), (32, 32, 64)])
def test_views_create_rejects_bad_tiling(tiling):
    with pytest.raises(abi.PGError) as e:
        abi.pg_views_create([_cam()], 1, 10, 0, abi.make_tiling(*tiling))
    assert e.value.status == -1


def test_views_create_rejects_bad_sh_degree_and_overflow():
    with pytest.raises(abi.PGError):
        abi.pg_views_create([_cam()], 1, 10, 4, abi.make_tiling())
    with pytest.raises(abi.PGError) as e:
        abi.pg_views_create([_cam()] * 3, 1, 2 ** 30, 0, abi.make_tiling())
    assert "2^31" in str(e.value)
    with pytest.raises(abi.PGError) as e:     # one projection grid row per frame
        abi.pg_views_create([_cam()], 65536, 10, 0, abi.make_tiling())
    assert "frames must be" in str(e.value)


def test_entry_points_reject_null_pointers():
    lib = abi.lib()
    assert lib.pg_loss_l1(None, None, 10, None, None, None, None) == -1
    assert "null" in abi.pg_last_error()
    assert lib.pg_adam_step(None, None, None, None, None, None, 1, 1, 1, 1, 1, 0.1, 0.9, 0.99, 1e-8, 1, None, None) == -1
    n = C.c_size_t()
    assert lib.pg_fetch_workspace_size(0, 5, C.byref(n)) == -1
    assert lib.pg_fetch_workspace_size(64, 64, C.byref(n)) == 0 and n.value > 0


def test_fake_quant_rejects_bad_arguments_on_the_host():
    """Widths outside [0, 16], too many channels and missing buffers are
    refused before any device work (the pointers below are never touched)."""
    lib = abi.lib()
    dummy = C.c_void_p(0x1000)
    bits = (C.c_int32 * 3)(8, 17, 8)
    assert lib.pg_atlas_fake_quant(dummy, dummy, 4, 1, 3, C.cast(bits, C.c_void_p), dummy, None, dummy, None) == -1
    assert "bits" in abi.pg_last_error()
    ok = (C.c_int32 * 3)(8, 8, 8)
    assert lib.pg_atlas_fake_quant(dummy, dummy, 4, 1, 3, C.cast(ok, C.c_void_p), None, None, dummy, None) == -1
    assert "null" in abi.pg_last_error()
    many = (C.c_int32 * 65)(*([8] * 65))
    assert lib.pg_atlas_fake_quant(dummy, dummy, 4, 1, 65, C.cast(many, C.c_void_p), dummy, None, dummy, None) == -1
    assert abi.lpo_bits(59) == [16, 16, 16] + [8] * 56


def test_new_boundary_calls_reject_bad_arguments_on_the_host():
    """pg_status_check, pg_workspace_query and pg_backward refuse null
    arguments before any device work (the dummy pointers are never read)."""
    lib = abi.lib()
    need = C.c_int64(-7)
    assert lib.pg_status_check(None, None, C.byref(need), None) == -1
    assert "null" in abi.pg_last_error() and need.value == -7
    plan = abi.pg_plan()
    assert lib.pg_workspace_query(None, 64, 64, 1000, C.byref(plan)) == -1
    args = [None] * 26
    args[10], args[20], args[21], args[24] = 0, 1, 1, 0
    assert lib.pg_backward(*args) == -1
    assert "null" in abi.pg_last_error()


def test_fetch_noalloc_refuses_atlases_beyond_its_scratch_on_the_host():
    """The allocation-free fetch refuses null buffers and atlases larger than
    its fixed scratch serves before any device work (the dummy pointers are
    never read), and its documented limit fits the workspace that
    pg_atlas_fetch would need at that size."""
    lib = abi.lib()
    dummy = C.c_void_p(0x1000)
    assert lib.pg_atlas_fetch_noalloc(None, dummy, 1, 14, 64, 64, 10, dummy, dummy, dummy, dummy, None) == -1
    assert "null" in abi.pg_last_error()
    assert lib.pg_atlas_fetch_noalloc(dummy, dummy, 1, 14, 8192, 8193, 10, dummy, dummy, dummy, dummy, None) == -5
    assert str(abi.FETCH_NOALLOC_MAX_TEXELS) in abi.pg_last_error()
    assert abi.pg_fetch_workspace_size(8192, 8192) <= abi.FETCH_NOALLOC_SCRATCH_BYTES
    src = open(os.path.join(ROOT, "include", "packuv_gs.h")).read()
    assert "#define PG_FETCH_NOALLOC_MAX_TEXELS (1LL << 26)" in src
    assert "#define PG_FETCH_NOALLOC_SCRATCH_BYTES (256u * 1024u)" in src
