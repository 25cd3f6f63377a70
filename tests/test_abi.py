"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point that include/etc.h declares,
and reject bad arguments before touching the device.
"""

import ctypes
import os
import re

import pytest

import paper_2404_02433_amd as etc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(etc_[A-Za-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = etc.load_library()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps every exported entry point with the same name
    for name in names:
        assert name in etc._SYMBOLS, name


def test_version_and_defaults():
    assert "gfx950" in etc.etc_version()
    o = etc._options()
    assert o.rtol == 1e-6 and o.max_iter == 1000 and o.refine_every == 20
    assert o.precision == 0 and o.kref_mode == 0


def test_workspace_size_scales_with_precision():
    b64 = etc.etc_workspace_size((64, 64, 64), "float64", 0)
    b32 = etc.etc_workspace_size((64, 64, 64), "float64", 0, precision="mixed")
    V = 64 ** 3
    # FP64: kappa, p, r, w, q, t = 6 doubles per voxel (+ tables)
    assert 48 * V <= b64 < 49 * V
    # mixed with float64 input: kappa32, kappa64, p64, r, w, q, t and the
    # solution increment (float32)
    assert 40 * V <= b32 < 41 * V
    b32in = etc.etc_workspace_size((64, 64, 64), "float32", 0, precision="mixed")
    assert 32 * V <= b32in < 33 * V


@pytest.mark.parametrize("shape,axis", [((0, 4, 4), 0), ((1, 4, 4), 0), ((4, 4, 4), 3), ((4, 1, 4), 1),
                                        ((4, 4, 4000), 2)])
def test_workspace_size_rejects_bad_shapes(shape, axis):
    with pytest.raises(etc.EtcError) as e:
        etc.etc_workspace_size(shape, "float64", axis)
    assert e.value.status in (-1, -6)


def test_mixed_form_load_axis_limit():
    """The mixed form's guarded tridiagonal partitions hold at most 16 rows
    (load axes up to 512); the float64 form goes to 2048."""
    etc.etc_workspace_size((512, 4, 4), "float32", 0, precision="mixed")
    etc.etc_workspace_size((2048, 4, 4), "float64", 0)
    with pytest.raises(etc.EtcError) as e:
        etc.etc_workspace_size((513, 4, 4), "float32", 0, precision="mixed")
    assert e.value.status == -6


def test_setup_rejects_bad_arguments_without_device():
    lib = etc.load_library()
    n = (ctypes.c_int64 * 3)(4, 4, 4)
    o = etc._options()
    h = ctypes.c_void_p(0)
    # NULL kappa
    assert lib.etc_setup(None, 0, n, etc._BC(1.0, 0.0), 0, ctypes.byref(o), ctypes.byref(h)) == -1
    assert "kappa" in etc.etc_last_error()
    # p_in == p_out: no potential drop, K_eff undefined
    fake = ctypes.c_void_p(0x1000)
    assert lib.etc_setup(fake, 0, n, etc._BC(1.0, 1.0), 0, ctypes.byref(o), ctypes.byref(h)) == -1
    assert "p_in" in etc.etc_last_error()
    # bad axis, bad rtol, bad dtype
    assert lib.etc_setup(fake, 0, n, etc._BC(1.0, 0.0), 5, ctypes.byref(o), ctypes.byref(h)) == -1
    o.rtol = 0.0
    assert lib.etc_setup(fake, 0, n, etc._BC(1.0, 0.0), 0, ctypes.byref(o), ctypes.byref(h)) == -1
    o = etc._options()
    assert lib.etc_setup(fake, 7, n, etc._BC(1.0, 0.0), 0, ctypes.byref(o), ctypes.byref(h)) == -1
    # mixed-sign domain lengths
    o = etc._options(L=(1.0, 0.0, 1.0))
    assert lib.etc_setup(fake, 0, n, etc._BC(1.0, 0.0), 0, ctypes.byref(o), ctypes.byref(h)) == -1
    assert h.value in (None, 0)


def test_state_errors_on_null_plan():
    lib = etc.load_library()
    d = ctypes.c_double()
    assert lib.etc_keff(None, ctypes.byref(d), None, None) == -1
    assert lib.etc_solve(None, None, None) == -1
    assert lib.etc_set_kernel_timer(None, 1) == -1
    lib.etc_destroy(None)  # no-op


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits
    before touching a device."""
    import json
    import subprocess
    import sys

    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]


def _static_call(shape, opts=None, k_out=True):
    lib = etc.load_library()
    o = etc._options(**(opts or {}))
    ko, ki = ctypes.c_double(0.0), ctypes.c_double(0.0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first
    return lib.etc_solve_static(fake, 0, etc._dims(shape), etc._BC(1.0, 0.0), 0, ctypes.byref(o), None,
                                ctypes.byref(ko) if k_out else None, ctypes.byref(ki), None)


def test_static_entry_rejects_before_touching_the_device():
    # beyond the static scratch array (128^3 float64 needs about 96 MiB)
    assert etc.etc_workspace_size((128, 128, 128), "float64", 0) > etc.STATIC_SCRATCH_BYTES
    assert _static_call((128, 128, 128)) == -6
    assert "scratch" in etc.etc_last_error()
    # a caller workspace, the autotuner, graphs or the adjoint are refused
    assert _static_call((16, 16, 16), {"autotune": True}) == -1
    assert _static_call((16, 16, 16), {"use_graph": True}) == -1
    assert _static_call((16, 16, 16), {"want_grad": True}) == -1
    assert _static_call((16, 16, 16), k_out=False) == -1
    assert _static_call((1, 16, 16)) == -1
    # the largest float64 cube the array holds
    assert etc.etc_workspace_size((96, 96, 96), "float64", 0) <= etc.STATIC_SCRATCH_BYTES


def test_ensemble_sizing_and_limits():
    shapes = [(48, 48, 48), (64, 64, 64), (48, 48, 48)]
    total = etc.etc_workspace_size_ensemble(shapes, "float32", 0, precision="mixed")
    per = etc.etc_workspace_size((48, 48, 48), "float32", 0, precision="mixed")
    # one batch workspace per shape (a batch shares its tables, so slightly under the sum of singles)
    assert 0.99 * (2 * per + etc.etc_workspace_size((64, 64, 64), "float32", 0, precision="mixed")) <= total
    # at most 8 distinct shapes, load axes up to 512, each shape valid
    with pytest.raises(etc.EtcError) as e:
        etc.etc_workspace_size_ensemble([(8 + i, 8, 8) for i in range(9)], "float64", 0)
    assert e.value.status == -6
    with pytest.raises(etc.EtcError) as e:
        etc.etc_workspace_size_ensemble([(600, 8, 8)], "float64", 0)
    assert e.value.status == -6
    with pytest.raises(etc.EtcError) as e:
        etc.etc_workspace_size_ensemble([(1, 8, 8)], "float64", 0)
    assert e.value.status == -1
