"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/gsr.h declares, and its defaults match the
oracle's reading of the renderer constants; and the exactness in bf16 of
the per-pixel columns the backward contraction feeds its matrix cores."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("gsr_create", "gsr_destroy", "gsr_plan", "gsr_render_forward", "gsr_render_backward",
                 "gsr_l1_loss_grad", "gsr_render_l1_fused", "gsr_graph_capture", "gsr_graph_launch",
                 "gsr_autotune", "gsr_check_overflow", "gsr_debug_tiles"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2311_11700_amd as gsr
    lib = gsr.load()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # The binding declares exactly the header's functions.
    assert sorted(gsr.exported_symbols()) == _declared_functions()


def test_struct_layouts():
    from paper_2311_11700_amd import _abi as A
    assert ctypes.sizeof(A.gsr_camera) == 80
    assert ctypes.sizeof(A.gsr_gaussians) == 8 + 7 * 8
    assert ctypes.sizeof(A.gsr_config) == 44
    assert ctypes.sizeof(A.gsr_images) == 40
    assert ctypes.sizeof(A.gsr_grads) == 56
    assert ctypes.sizeof(A.gsr_tuning) == 16
    assert ctypes.sizeof(A.gsr_gaussians_out) == 6 * 8


def test_defaults_match_oracle_constants():
    import numpy as np

    import oracle as O
    import paper_2311_11700_amd as gsr
    c = gsr.load().gsr_default_config()
    o = O.Config().as_f32()
    assert c.alpha_min == o.alpha_min and c.alpha_max == o.alpha_max and c.T_min == o.T_min
    assert c.cutoff_sigma == o.cutoff and c.z_near == o.z_near and c.lowpass == o.lowpass
    assert list(c.bg) == [0.0, 0.0, 0.0]
    assert c.flags == gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD
    assert c.fov_guard == o.fov_guard == np.float32(gsr.Config().fov_guard)
    assert np.float32(gsr.Config().alpha_min) == np.float32(c.alpha_min)


def test_status_strings_and_null_context():
    import paper_2311_11700_amd as gsr
    lib = gsr.load()
    for st in (0, -1, -2, -3, -4, -5):
        assert lib.gsr_status_string(st)
    assert lib.gsr_plan(None, 10, 1, None, 100, None) == gsr.GSR_E_INVALID
    assert lib.gsr_last_error(None) == b"null context"


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2311_11700_amd import _abi as A
    monkeypatch.setattr(A, "_LIB", None)
    monkeypatch.setattr(A, "LIB_PATH", "/nonexistent/libgsr.so")
    with pytest.raises(RuntimeError, match="no fallback"):
        A.load()


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2311_11700_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_backward_contraction_operands_fit_bf16():
    """The fused backward's matrix-core contraction takes its per-pixel
    columns in bf16 without rounding: the moment polynomials 1, x, y, x^2,
    x y, y^2 of the tile-centred pixel coordinates (half-integers from -7.5
    to 7.5) and the L1 residual signs.  bf16 keeps the top 16 bits of a
    float32, so exactness means the low 16 bits are zero; a value with more
    than 8 significant bits (e.g. 7.5 * 7.5 + 1/8) would not pass."""
    c = np.arange(16, dtype=np.float64) - 7.5
    x, y = np.meshgrid(c, c)
    cols = [np.ones_like(x), x, y, x * x, x * y, y * y, np.array([-1.0, 0.0, 1.0])]
    for v in cols:
        f = np.asarray(v, np.float32)
        assert np.array_equal(f.astype(np.float64), np.asarray(v, np.float64))
        assert not (f.view(np.uint32) & 0xFFFF).any()
    assert np.float32(7.5 * 7.5 + 0.125).view(np.uint32) & 0xFFFF
