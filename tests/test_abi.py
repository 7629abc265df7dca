"""CPU checks of the C ABI: the library loads, exports every function that
include/gg.h declares, its structs have the layout the binding assumes, and
argument validation rejects bad calls before anything reaches the GPU."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gg.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2511_10353_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2511_10353_amd import build
        build.build(verbose=False)
    return binding.lib()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for want in ("gg_noise", "gg_filter", "gg_fft3d", "gg_zeldovich", "gg_make_ic", "gg_plan_create"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    nm = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (gg_\w+)", nm))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing


def test_struct_layout_matches_binding(tmp_path):
    from paper_2511_10353_amd import binding
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "gg.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(gg_grid), offsetof(gg_grid, box), sizeof(gg_cosmo));
  printf("%zu %zu %zu\n", offsetof(gg_cosmo, amp), offsetof(gg_cosmo, lattice_offset), sizeof(gg_plan_info));
  printf("%zu %zu %zu %zu\n", offsetof(gg_plan_info, box), offsetof(gg_plan_info, real_elems),
         offsetof(gg_plan_info, workspace_bytes), offsetof(gg_plan_info, chunks));
  printf("%zu %zu\n", offsetof(gg_plan_info, p1_lines), offsetof(gg_plan_info, z_lines));
  printf("%zu %zu %zu\n", sizeof(gg_tune_entry), offsetof(gg_tune_entry, ms), sizeof(gg_zoom_desc));
  printf("%zu %zu %zu\n", offsetof(gg_zoom_desc, origin), offsetof(gg_zoom_desc, box), offsetof(gg_zoom_desc, variant));
  printf("%zu %zu\n", sizeof(gg_zoom_tune_entry), offsetof(gg_zoom_tune_entry, ms));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(binding._Grid), binding._Grid.box.offset, ctypes.sizeof(binding._Cosmo),
            binding._Cosmo.amp.offset, binding._Cosmo.lattice_offset.offset, ctypes.sizeof(binding._Info),
            binding._Info.box.offset, binding._Info.real_elems.offset, binding._Info.workspace_bytes.offset,
            binding._Info.chunks.offset, binding._Info.p1_lines.offset, binding._Info.z_lines.offset,
            ctypes.sizeof(binding._TuneEntry), binding._TuneEntry.ms.offset, ctypes.sizeof(binding._ZoomDesc),
            binding._ZoomDesc.origin.offset, binding._ZoomDesc.box.offset, binding._ZoomDesc.variant.offset,
            ctypes.sizeof(binding._ZoomTuneEntry), binding._ZoomTuneEntry.ms.offset]
    assert got == want


def test_status_strings(lib):
    for code, name in [(0, b"GG_OK"), (1, b"GG_ERR_INVALID_ARG"), (2, b"GG_ERR_UNSUPPORTED_SIZE"),
                       (3, b"GG_ERR_OUT_OF_MEMORY"), (4, b"GG_ERR_HIP"), (5, b"GG_ERR_INTERNAL")]:
        assert lib.gg_status_string(code) == name


def _create(lib, n=32, box=100.0, dtype=0, **kw):
    from paper_2511_10353_amd import binding
    h = ctypes.c_void_p()
    cosmo = binding.Cosmo(**kw)._c()
    st = lib.gg_plan_create(ctypes.byref(h), ctypes.byref(binding._Grid(n, box)), ctypes.byref(cosmo), dtype)
    return st, lib.gg_last_error().decode()


@pytest.mark.parametrize("n", [0, 7, 12, 48, 100, 2048, -8])
def test_unsupported_sizes_rejected(lib, n):
    st, msg = _create(lib, n=n)
    assert st == 2 and "power of two" in msg


@pytest.mark.parametrize("kw,box,dtype", [({}, 0.0, 0), ({}, -1.0, 0), ({}, float("inf"), 0), ({}, 100.0, 2),
                                          ({"omega_m": 0.0}, 100.0, 0), ({"h": -0.7}, 100.0, 0),
                                          ({"z_init": -1.0}, 100.0, 0), ({"sigma8": 0.0}, 100.0, 0),
                                          ({"amp": -1.0}, 100.0, 0), ({"lattice_offset": float("nan")}, 100.0, 0),
                                          ({"lattice_offset": 1.0}, 100.0, 0), ({"lattice_offset": -0.25}, 100.0, 0),
                                          ({"lattice_offset": 1024.5}, 100.0, 1)])
def test_bad_arguments_rejected(lib, kw, box, dtype):
    st, msg = _create(lib, box=box, dtype=dtype, **kw)
    assert st == 1 and msg


def test_null_arguments_rejected(lib):
    assert lib.gg_plan_create(None, None, None, 0) == 1
    assert lib.gg_workspace_bytes(None) == 0
    assert lib.gg_noise(None, 1, 0, None, None) == 1
    assert lib.gg_fft3d(None, 1, None, None, None, None) == 1
    assert lib.gg_filter(None, None, None, None, None) == 1
    assert lib.gg_zeldovich(None, None, None, None, None) == 1
    assert lib.gg_make_ic(None, 1, None, None, None, None, None) == 1
    assert lib.gg_plan_query(None, None) == 1
    assert lib.gg_timing_enable(None, 1) == 1
    assert lib.gg_plan_destroy(None) == 0


@pytest.mark.parametrize("n,box,r_s", [(32, 100.0, 2 * 100.0 / 16), (64, 300.0, 2 * 300.0 / 32), (48, 40.0, 0.8),
                                       (32, 2 * 3.14159265358979323846 * 3.0, 1.0)])
def test_cutoff_n2_selects_the_oracle_large_scale_window(lib, n, box, r_s):
    # host-only call: the modes with n^2 < cutoff are exactly those the
    # oracle's top hat f(k r_s) = [k r_s < 1] keeps (Eq. 4-5)
    from oracle import pipeline, refine
    cut = lib.gg_cutoff_n2(box, r_s)
    s = pipeline.signed_index(n)
    n2 = s.reshape(n, 1, 1) ** 2 + s.reshape(1, n, 1) ** 2 + np.arange(n // 2 + 1).reshape(1, 1, -1) ** 2
    assert np.array_equal(n2 < cut, refine.mode_window(n, box, r_s, "large") > 0)
    assert lib.gg_cutoff_n2(0.0, 1.0) == -1 and lib.gg_cutoff_n2(100.0, float("nan")) == -1


def test_increase_resolution_validates_before_touching_the_gpu(lib):
    assert lib.gg_increase_resolution(None, None, None, 2, 0, 1, 0.0, None, None, None, None) == 1


def test_out_of_range_enums_rejected(lib):
    # a C caller may pass any int for an enum parameter: rejected, not used
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert lib.gg_refine_noise(16, 7, 2, fake, 1, 1, fake, None) == 1
    assert lib.gg_refine_noise(16, 0, 9, fake, 1, 1, fake, None) == 1
    origin = (ctypes.c_int32 * 3)(0, 0, 0)
    assert lib.gg_refine_noise_region(16, origin, 8, 2, 2, fake, 1, 1, fake, None) == 1
    assert lib.gg_interpolate_add(8, 16, 5, fake, fake, None) == 1
    assert lib.gg_interpolate_add_at(8, 2, origin, 8, -1, fake, fake, None) == 1
    st, msg = _create(lib, dtype=-3)
    assert st == 1 and "dtype" in msg
