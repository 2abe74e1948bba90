"""The C ABI on the CPU: the library loads, exports every declared entry point,
and validates its arguments before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1603_03590_amd import _lib, params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dis.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dis_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_params_struct_layout_matches_header():
    # double fields are 8-byte aligned: 4+4(pad)+8 +4*5 +4(pad) +8*4 +4+4 +4+4(pad)+8 = 96
    assert ctypes.sizeof(_lib.dis_params) == 96


@pytest.mark.parametrize("preset", [1, 2, 3, 4, 101, 102, 103, 104, 105, 106])
def test_presets(preset):
    p = params(preset)
    assert p.patch_size in (8, 12)
    assert p.w_intensity == 5.0 and p.w_gradient == 10.0 and p.w_smooth == 10.0
    assert p.var_inner == 5


def test_paper_operating_points():
    """Sec. 3.3: the four operating points, with theta_ss 5."""
    ops = {1: (3, 16, 8, 0.3, 0), 2: (3, 12, 8, 0.4, 1), 3: (1, 16, 12, 0.75, 1), 4: (0, 256, 12, 0.75, 1)}
    for k, (sf, it, ps, ov, ref) in ops.items():
        p = params(k)
        assert (p.finest_scale, p.gn_iters, p.patch_size, p.overlap, p.refine) == (sf, it, ps, ov, ref)
        assert p.coarsest_scale == 5 and p.var_outer == -1


def test_unknown_preset():
    with pytest.raises(_lib.DisError) as e:
        params(77)
    assert e.value.code == _lib.DIS_EINVAL


@pytest.mark.parametrize("field,value", [
    ("patch_size", 7), ("patch_size", 2), ("patch_size", 18), ("overlap", 1.0), ("overlap", -0.1),
    ("finest_scale", -1), ("coarsest_scale", -2), ("gn_iters", -1), ("var_inner", 0),
    ("sor_omega", 2.0), ("sor_omega", 0.0), ("w_smooth", -1.0), ("refine", 2), ("flags", 0x100),
])
def test_create_rejects_bad_params(field, value):
    p = params(2, **{field: value})
    with pytest.raises(_lib.DisError) as e:
        _lib.dis_create(p, 64, 64)
    assert e.value.code == _lib.DIS_EINVAL
    assert _lib.dis_last_error()


def test_create_rejects_bad_sizes():
    with pytest.raises(_lib.DisError) as e:
        _lib.dis_create(params(2), 64, 64, 0)
    assert e.value.code == _lib.DIS_EINVAL
    with pytest.raises(_lib.DisError) as e:
        _lib.dis_create(params(2, finest_scale=3), 32, 32)     # 4x4 at scale 3 < 8 px patch
    assert e.value.code == _lib.DIS_ESIZE
    with pytest.raises(_lib.DisError) as e:
        _lib.dis_create(params(2, finest_scale=4, coarsest_scale=3), 512, 512)
    assert e.value.code == _lib.DIS_EINVAL


def test_null_handles():
    lib = _lib.load()
    assert lib.dis_compute_flow(None, None, None, 8, 8, 8, None) == _lib.DIS_EINVAL
    assert lib.dis_flow_backward(None, None, None, None) == _lib.DIS_EINVAL
    assert lib.dis_set_stream(None, None) == _lib.DIS_EINVAL
    assert lib.dis_debug_level(None, 0, 0, None, 0) == _lib.DIS_EINVAL
    assert lib.dis_compute_flow_batched(None, 0, None, None, None, None, None, None) == _lib.DIS_EINVAL
    assert lib.dis_default_params(1, None) == _lib.DIS_EINVAL
    assert lib.dis_create(None, 8, 8, 1, None, None) == _lib.DIS_EINVAL
    lib.dis_destroy(None)                      # NULL is ignored
    assert _lib.dis_last_error()


def test_noalloc_call_checks_arguments_before_any_hip_call():
    lib = _lib.load()
    assert lib.dis_compute_flow_noalloc(None, None, None, 8, 8, 8, None, None) == _lib.DIS_EINVAL
    p = params(102)
    assert lib.dis_compute_flow_noalloc(ctypes.byref(p), None, None, 1024, 436, 1024, None, None) == _lib.DIS_EINVAL
    p = params(105, flags=_lib.DIS_FLAG_COLOUR)
    assert lib.dis_compute_flow_noalloc(ctypes.byref(p), 1, 1, 512, 256, 512, 1, None) == _lib.DIS_EINVAL
    assert "DIS_FLAG_COLOUR" in _lib.dis_last_error()
    p = params(102)
    assert lib.dis_compute_flow_noalloc(ctypes.byref(p), 1, 1, 1024, 436, 1000, 1, None) == _lib.DIS_EINVAL
    assert lib.dis_compute_flow_noalloc(ctypes.byref(p), 1, 1, 40, 40, 40, 1, None) == _lib.DIS_ESIZE


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1603_03590_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
