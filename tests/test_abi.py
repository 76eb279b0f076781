"""CPU checks of the C ABI: the library loads, exports every symbol that
include/lar.h declares, and rejects bad arguments on the host (no GPU work)."""
import ctypes
import os
import re

import pytest

from paper_2203_02479_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lar.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lar_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lar():
    from paper_2203_02479_amd import lar as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("liblar.so not built")
    return L


def test_every_declared_symbol_is_exported_and_bound(lar):
    syms = declared_symbols()
    assert len(syms) >= 10
    L = lar.lib()
    for s in syms:
        assert hasattr(L, s), s
        assert s in lar.SIGNATURES, s


def test_status_strings(lar):
    L = lar.lib()
    for code in (0, -1, -2, -3, -4):
        assert L.lar_status_str(code)
    assert L.lar_status_str(7) == b"unknown status"


def test_workspace_queries_and_size_checks(lar):
    P = inputs.cfg1_plane()
    ld = (3073 + 15) // 16 * 16
    assert lar.fftconv_workspace(P) == 4800 * ld * 8 + (480 * ld * 8 + 255) // 256 * 256
    assert lar.sim_plane_workspace(P) == 4800 * 6000 * 4 + lar.fftconv_workspace(P)
    assert lar.raster_workspace(P, 1000, None) == 0
    fixed = 256 + ((1000 + 15) // 16 + 255) // 256 * 256
    assert lar.raster_workspace(P, 1000, (1, 0, 0, 0)) == fixed + (1000 * 16 + 4096) * 24
    assert (lar.sim_plane_workspace(P, 1000, (2, 0, 0, 0))
            == lar.sim_plane_workspace(P) + lar.raster_workspace(P, 1000, (2, 0, 0, 0)))
    for bad in (dict(nt_fft=6000 + 2 * 7), dict(nt_fft=5999), dict(nw_fft=500), dict(nw_fft=400),
                dict(nt_fft=32768), dict(nw_fft=1152)):
        Q = inputs.cfg1_plane()
        for k, v in bad.items():
            setattr(Q, k, v)
        with pytest.raises(lar.LarError) as e:
            lar.fftconv_workspace(Q)
        assert e.value.status == lar.LAR_ESIZE


def test_host_side_argument_errors(lar):
    L = lar.lib()
    P = lar.make_plane(inputs.cfg0_plane())
    d = lar.lar_depos(None, None, None, None, None, -1)
    R = L.lar_raster
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, None, None, None, 0, None) == lar.LAR_EINVAL
    d = lar.lar_depos(None, None, None, None, None, 0)
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, None, None, None, 0, None) == lar.LAR_OK
    assert R(ctypes.byref(P), ctypes.byref(d), 0.0, None, None, None, 0, None) == lar.LAR_EINVAL
    assert R(None, ctypes.byref(d), 3.0, None, None, None, 0, None) == lar.LAR_EINVAL
    f = lar.lar_fluct(3, 0, 0, 0, 0)
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, ctypes.byref(f), None, None, 0, None) == lar.LAR_EINVAL
    f = lar.lar_fluct(1, 0, 300, 0, 0)
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, ctypes.byref(f), None, None, 0, None) == lar.LAR_EINVAL
    one = ctypes.c_void_p(256)
    d = lar.lar_depos(one, one, one, one, one, 10)
    f = lar.lar_fluct(1, 0, 0, 0, 0)
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, ctypes.byref(f), one, None, 0, None) == lar.LAR_EWORKSPACE
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, ctypes.byref(f), one, one, 255, None) == lar.LAR_EWORKSPACE
    assert L.lar_fftconv(ctypes.byref(P), None, None, None, None, 0, None) == lar.LAR_EINVAL
    one = ctypes.c_void_p(256)
    assert L.lar_fftconv(ctypes.byref(P), one, one, one, None, 0, None) == lar.LAR_EWORKSPACE
    assert L.lar_fftconv(ctypes.byref(P), one, one, one, one, 16, None) == lar.LAR_EWORKSPACE
    assert L.lar_sample_counts(0, 1, one, one, one, 0, 0, one, None) == lar.LAR_EINVAL
    assert L.lar_sample_counts(1, 0, None, None, None, 0, 0, None, None) == lar.LAR_OK
