"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, fills defaults, and rejects invalid parameters before touching HIP."""
import math
import os
import re

import pytest

from paper_1903_06555_amd import wsp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "wsp.h")).read()
    return sorted(set(re.findall(r"\b(wsp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = wsp.load_library()
    names = _declared()
    assert "wsp_degrid" in names and "wsp_grid" in names and "wsp_build_kernels" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(wsp.EXPORTED) == names


def test_default_params():
    p = wsp.wsp_default_params()
    assert p.oversample == 2.0 and p.kb_support == 4 and p.n_stacks == 1
    assert p.quad_rel_tol == 1e-6 and p.quad_abs_tol == 1e-6
    assert p.kmeans_tol == 1e-3 and p.precision == wsp.WSP_FP32_FP64PHASE


@pytest.mark.parametrize("field,value", [
    ("n", 63), ("n", 0), ("oversample", 0.5), ("fov_rad", 0.0), ("fov_rad", 0.6),
    ("kb_support", 3), ("support_scale", 0.5), ("n_stacks", 0), ("fold_conjugate", 2),
    ("quad_max_panels", 4), ("quad_max_panels", 5000), ("precision", 7), ("kmeans_max_iter", 0),
    ("max_support", 2), ("kernel_mode", 7), ("plane_dq", -1.0), ("plane_dq", 2.0),
    ("plane_dw", float("nan")), ("dde_support", 2), ("dde_support", 17), ("dde_support", -1),
    ("item_taps", -1), ("item_taps", (1 << 24) + 1), ("band_rows", 4), ("band_rows", 32),
    ("tap_layout", -1), ("tap_layout", 3),
])
def test_create_rejects_invalid_parameters(field, value):
    p = wsp.make_params(64, math.radians(10.0))
    setattr(p, field, value)
    with pytest.raises(wsp.WspError) as ei:
        wsp.wsp_create(p)
    assert ei.value.status == wsp.WSP_EINVAL
    assert wsp.wsp_last_error()


def test_plane_mode_needs_fp32_path():
    p = wsp.make_params(64, math.radians(10.0), precision="fp64", kernels="planes")
    with pytest.raises(wsp.WspError) as ei:
        wsp.wsp_create(p)
    assert ei.value.status == wsp.WSP_EINVAL


def test_dde_needs_stored_kernels():
    p = wsp.make_params(64, math.radians(10.0), kernels="planes", dde_support=3)
    with pytest.raises(wsp.WspError) as ei:
        wsp.wsp_create(p)
    assert ei.value.status == wsp.WSP_EINVAL


@pytest.mark.parametrize("struct", [wsp.wsp_params, wsp.wsp_plan_info])
def test_struct_layout_matches_header(tmp_path, struct):
    """ctypes mirrors of the ABI structs have the C structs' sizes and field offsets."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    name = struct.__name__
    fields = [f for f, _ in struct._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"wsp.h\"\nint main(void){\n"
                   f"printf(\"%zu\\n\", sizeof({name}));\n" +
                   "".join(f"printf(\"%zu\\n\", offsetof({name}, {f}));\n" for f in fields) +
                   "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(struct)
    assert out[1:] == [getattr(struct, f).offset for f in fields]


def test_grid_side_must_tile():
    p = wsp.make_params(48, math.radians(10.0))   # G = 96 is not a multiple of 64
    with pytest.raises(wsp.WspError):
        wsp.wsp_create(p)


def test_null_arguments():
    lib = wsp.load_library()
    assert lib.wsp_create(None, None) == wsp.WSP_EINVAL
    assert lib.wsp_footprint(None, None, None, None) == wsp.WSP_EINVAL
    assert lib.wsp_degrid(None, None, None, None) == wsp.WSP_EINVAL
    lib.wsp_destroy(None)
