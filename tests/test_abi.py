"""Host-side checks of the C-ABI library (no GPU needed): the library loads,
exports every entry point declared in include/ebit.h, sizes workspaces and
rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ebit.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(ebit_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("ebit_workspace_bytes", "ebit_create", "ebit_advect", "ebit_fraction", "ebit_curvature",
              "ebit_fraction_curvature", "ebit_get_state", "ebit_set_state", "ebit_stats", "ebit_sync",
              "ebit_destroy", "ebit_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2309_00338_amd import ebit

    lib = ctypes.CDLL(ebit.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_workspace_bytes_and_argument_errors():
    from paper_2309_00338_amd import ebit

    b64 = ebit.workspace_bytes(64, 64, 1 / 64)
    b128 = ebit.workspace_bytes(128, 128, 1 / 128)
    # two copies of colours (bytes) and offsets (FP64) dominate
    assert 2 * (65 * 65 + 64 * 64 + 8 * 2 * 64 * 65) <= b64 < 2 * b64
    assert 3.5 * b64 < b128 < 4.5 * b64
    with pytest.raises(ebit.EbitError) as e:
        ebit.workspace_bytes(3, 64, 1 / 64)
    assert e.value.code == ebit.EBIT_ERR_ARG
    with pytest.raises(ebit.EbitError):
        ebit.workspace_bytes(64, 64, -1.0)
    with pytest.raises(ebit.EbitError):
        ebit.workspace_bytes(64, 64, 1 / 64, flags=8)
    lib = ebit.lib()
    # create with a null workspace or null state fails before any device call
    g = ebit.ebit_grid(16, 16, 1 / 16, 0)
    h = ctypes.c_void_p()
    assert lib.ebit_create(ctypes.byref(g), None, None, 0, None, ctypes.byref(h)) == ebit.EBIT_ERR_ARG
    for fn in ("ebit_advect", "ebit_fraction", "ebit_sync", "ebit_destroy", "ebit_stats_reset"):
        f = getattr(lib, fn)
        nargs = len(f.argtypes)
        args = [None] * nargs
        if fn == "ebit_advect":
            args[-1] = 0.1
        assert f(*args) == ebit.EBIT_ERR_ARG, fn
    assert ebit.strerror(ebit.EBIT_ERR_CFL).startswith("a marker moved")


def test_create_rejects_out_of_range_state_on_host():
    from paper_2309_00338_amd import ebit, inputs

    st = inputs.init_state(16, 16, [inputs.Circle(8.2, 7.9, 4.1)])
    lib = ebit.lib()
    g = ebit.ebit_grid(16, 16, 1 / 16, 0)
    h = ctypes.c_void_p()
    bad = st.copy()
    hp = bad.h_present()
    jj, ii = np.nonzero(hp)
    bad.hoff[jj[0], ii[0]] = 1.5
    s, keep = ebit._host_state(bad)
    ws = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert lib.ebit_create(ctypes.byref(g), ctypes.byref(s), ws, 1 << 40, None, ctypes.byref(h)) == ebit.EBIT_ERR_ARG
    bad = st.copy()
    bad.c[3, 3] = 2
    s, keep = ebit._host_state(bad)
    assert lib.ebit_create(ctypes.byref(g), ctypes.byref(s), ws, 1 << 40, None, ctypes.byref(h)) == ebit.EBIT_ERR_ARG
