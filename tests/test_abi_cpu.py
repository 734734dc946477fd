"""Host-side checks of the C interface that need no GPU: the library loads and
exports every function include/gs.h declares; argument validation that
happens before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_interface():
    names = declared_functions()
    for must in ("gs_create", "gs_destroy", "gs_upload_scene", "gs_render_batch", "gs_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2510_15352_amd as gs
    lib = gs.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(gs.EXPORTS) | set(declared_functions())
    assert set(gs.EXPORTS) == set(declared_functions())


def test_null_context_and_bad_arguments_rejected_without_gpu():
    import paper_2510_15352_amd as gs
    lib = gs.load()
    assert lib.gs_destroy(None) == -1
    assert lib.gs_last_error(None) == b"null context"
    out = ctypes.c_void_p()
    assert lib.gs_create(0, None) == -1
    rc = lib.gs_render_batch(None, 1, None, None, None, 64, 48, None, None, None, None, None)
    assert rc == -1
    opts = gs.binding.RenderOpts()
    lib.gs_default_opts(ctypes.byref(opts))
    assert opts.near_plane == pytest.approx(0.2) and opts.mode == gs.GS_MODE_BATCHED
    assert opts.persistent == -1 and opts.use_graph == 0
    del out


def test_struct_layouts_match_library():
    import paper_2510_15352_amd as gs
    lib = gs.load()
    sizes = [ctypes.c_int32() for _ in range(3)]
    assert lib.gs_abi_sizes(*[ctypes.byref(s) for s in sizes]) == 0
    assert [s.value for s in sizes] == [ctypes.sizeof(gs.binding.SceneDesc),
                                        ctypes.sizeof(gs.binding.RenderOpts),
                                        ctypes.sizeof(gs.binding.Stats)]


def test_scaled_walk_constants():
    """The raster walk runs on alpha / 0.99 and 0.99 x the transmittance:
    its log2(0.99) literal and its scaled thresholds must come from the
    fixed rules (alpha clamp 0.99, skip below 1/255, stop under 1e-4)."""
    import numpy as np
    src = open(os.path.join(ROOT, "paper_2510_15352_amd", "csrc", "gs_device.h")).read()

    def const(name):
        return re.search(r"constexpr float %s = ([^;]+);" % name, src).group(1).strip()

    assert np.float32(const("kAlphaMax").rstrip("f")) == np.float32(0.99)
    assert const("kAlphaMin") == "1.0f / 255.0f"
    assert np.float32(const("kTMin").rstrip("f")) == np.float32(1e-4)
    assert const("kScaledAlphaMin") == "kAlphaMin / kAlphaMax"
    assert const("kScaledTMin") == "kTMin * kAlphaMax"
    assert np.float32(const("kLog2AlphaMax").rstrip("f")) == np.float32(np.log2(0.99))
