"""Host-side checks of the C-ABI library (no GPU needed): the library loads,
exports every entry point declared in include/*.h (ebit.h, ebit_film.h),
sizes workspaces and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", hdr)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"^\s*(?:int|const char \*)\s*(ebit_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("ebit_workspace_bytes", "ebit_create", "ebit_advect", "ebit_fraction", "ebit_curvature",
              "ebit_fraction_curvature", "ebit_get_state", "ebit_set_state", "ebit_stats", "ebit_sync",
              "ebit_destroy", "ebit_strerror"):
        assert n in names
    for n in ("ebit_film_workspace_bytes", "ebit_film_create", "ebit_film_advect", "ebit_film_fraction",
              "ebit_film_get_state", "ebit_film_set_state", "ebit_film_stats", "ebit_film_sync", "ebit_film_destroy"):
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
    # the fit-job list of one grid (2 directions x 8 queue regions of 256
    # entries per tile of a share) must stay within 32-bit indices: about
    # 46000^2 cells; beyond, the grid is refused rather than sized modulo 2^32
    big = ebit.workspace_bytes(46000, 46000, 1 / 46000)
    assert big > 8 * 2 * 46000 * 46001 * 2
    with pytest.raises(ebit.EbitError) as e:
        ebit.workspace_bytes(46400, 46400, 1 / 46400)
    assert e.value.code == ebit.EBIT_ERR_ARG
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


def test_film_workspace_and_host_validation():
    """The two-markers-per-edge entry points size their workspace and reject a
    bad grid, gap or state (a count of the wrong parity, three markers, offsets
    out of order or range) before any device call."""
    import math

    from paper_2309_00338_amd import ebit, film, inputs

    assert film.workspace_bytes(64, 64, 1 / 64) >= 2 * (65 * 65 + 64 * 64 + 2 * 16 * 64 * 65)
    with pytest.raises(ebit.EbitError):
        film.workspace_bytes(3, 64, 1 / 64)
    g = ebit.ebit_grid(16, 16, 1 / 16, 1)  # sweep-order flags are not supported
    n = ctypes.c_size_t()
    assert film._lib.ebit_film_workspace_bytes(ctypes.byref(g), ctypes.byref(n)) == ebit.EBIT_ERR_ARG
    st = film.FilmState.of(inputs.init_state(16, 16, [inputs.Circle(8.2, 7.9, 4.1)]))
    lib = film._lib
    g = ebit.ebit_grid(16, 16, 1 / 16, 0)
    h = ctypes.c_void_p()
    ws = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first

    def create(fs, delta=0.05):
        s, keep = fs._host()
        return lib.ebit_film_create(ctypes.byref(g), delta, ctypes.byref(s), 0, ws, 1 << 40, None, ctypes.byref(h))

    jj, ii = np.nonzero(st.hn)
    for edit in ("parity", "three", "order", "range"):
        bad = st.copy()
        j, i = jj[0], ii[0]
        if edit == "parity":
            bad.hn[j, i] = 2
            bad.ho[j, i] = (0.2, 0.6)
        elif edit == "three":
            bad.hn[j, i] = 3
        elif edit == "order":
            kk = np.nonzero(bad.hn == 0)
            bad.hn[kk[0][0], kk[1][0]] = 2
            bad.ho[kk[0][0], kk[1][0]] = (0.7, 0.3)
        else:
            bad.ho[j, i, 0] = 1.5
        assert create(bad) == ebit.EBIT_ERR_ARG, edit
    assert create(st, delta=-1.0) == ebit.EBIT_ERR_ARG
    assert create(st, delta=math.nan) == ebit.EBIT_ERR_ARG
    for fn in ("ebit_film_advect", "ebit_film_fraction", "ebit_film_sync", "ebit_film_destroy"):
        f = getattr(lib, fn)
        args = [None] * len(f.argtypes)
        if fn == "ebit_film_advect":
            args[-1] = 0.1
        assert f(*args) == ebit.EBIT_ERR_ARG, fn
