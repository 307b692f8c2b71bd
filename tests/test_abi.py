"""The C-ABI library loads and exports every entry point of include/pv3d.h (CPU only:
no GPU work is started here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pv3d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pv3d_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1410_5780_amd import pv3d
    if not os.path.exists(pv3d.LIB_PATH):
        from paper_1410_5780_amd import build
        build.build()
    return pv3d.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("pv3d_create", "pv3d_destroy", "pv3d_last_error", "pv3d_scene_load", "pv3d_scene_release",
                 "pv3d_generator_define", "pv3d_generator_release", "pv3d_sun_cooper", "pv3d_evaluate",
                 "pv3d_evaluate_batched", "pv3d_autotune", "pv3d_batch_stats", "pv3d_submit", "pv3d_poll",
                 "pv3d_wait", "pv3d_cancel", "pv3d_generator_define_tracked", "pv3d_generator_set_diode",
                 "pv3d_generator_set_sky", "pv3d_sky_view", "pv3d_profile_sample"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    from paper_1410_5780_amd import pv3d
    assert ctypes.sizeof(pv3d.Module) == 80
    assert ctypes.sizeof(pv3d.Params) == 24
    assert ctypes.sizeof(pv3d.Outputs) == 56
    assert ctypes.sizeof(pv3d.Job) == 136
    assert ctypes.sizeof(pv3d.Tracker) == 56
    assert ctypes.sizeof(pv3d.Diode) == 56


def test_sun_helper_matches_input_generator(lib):
    """Host helper (Cooper declination) against the numpy input generator."""
    from paper_1410_5780_amd import pv3d, workloads as W
    day = np.repeat(np.arange(1, 366, 7), 24)
    hour = np.tile(np.arange(24.0), day.size // 24)
    a = pv3d.sun_cooper(40.4, day, hour)
    b = W.cooper_sun(40.4, day, hour)
    assert np.max(np.abs(a - b)) < 1e-14


def test_errors_are_codes_not_crashes(lib):
    from paper_1410_5780_amd import pv3d
    h = ctypes.c_void_p()
    rc = lib.pv3d_create(0, 0, ctypes.byref(h))
    if rc == 0:                                  # a GPU is present: nothing more to check here
        lib.pv3d_destroy(h)
        return
    assert rc in (pv3d.EDEVICE, pv3d.EINVAL)
    assert len(lib.pv3d_last_error(None)) > 0
    assert lib.pv3d_create(0, 0, None) == pv3d.EINVAL
    lib.pv3d_destroy(None)
