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
    assert lar.raster_workspace(P, 1000, (1, 0, 0, 0)) == fixed + (1000 * 48 + 4096) * 16
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
    f = lar.lar_fluct(4, 0, 0, 0, 0)
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, ctypes.byref(f), None, None, 0, None) == lar.LAR_EINVAL
    f = lar.lar_fluct(3, 0, 0, 0, 0)
    assert R(ctypes.byref(P), ctypes.byref(d), 3.0, ctypes.byref(f), None, None, 0, None) == lar.LAR_OK
    # a fluctuated grid of 2^32 cells or more would wrap the bin counter word
    big = lar.make_plane(inputs.Plane(n_wires=1000, n_ticks=450000, n_imp=10, nt_fft=450000, nw_fft=1024))
    for mode in (1, 2, 3):
        f = lar.lar_fluct(mode, 0, 0, 0, 0)
        assert R(ctypes.byref(big), ctypes.byref(d), 3.0, ctypes.byref(f), None, None, 0, None) == lar.LAR_ESIZE
    f = lar.lar_fluct(0, 0, 0, 0, 0)
    assert R(ctypes.byref(big), ctypes.byref(d), 3.0, ctypes.byref(f), None, None, 0, None) == lar.LAR_OK
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
    assert L.lar_sample_counts(4, 1, one, one, one, 0, 0, one, None) == lar.LAR_EINVAL
    assert L.lar_sample_counts(1, 0, None, None, None, 0, 0, None, None) == lar.LAR_OK


def test_streams_host_side_errors(lar):
    L = lar.lib()
    P = lar.make_plane(inputs.cfg0_plane())
    pls = (lar.lar_plane * 1)(P)
    its = lar.make_items([(0, 0, 0, 0, 10, 0)])
    one = ctypes.c_void_p(256)
    nb = ctypes.c_size_t(0)
    assert L.lar_sim_streams_workspace(pls, 1, its, 1, None, 0, ctypes.byref(nb)) == lar.LAR_EINVAL
    assert L.lar_sim_streams_workspace(pls, 1, its, 1, None, 65, ctypes.byref(nb)) == lar.LAR_EINVAL
    assert L.lar_sim_streams_workspace(pls, 1, its, 1, None, 3, ctypes.byref(nb)) == lar.LAR_OK
    assert nb.value == 3 * lar.sim_plane_workspace(inputs.cfg0_plane(), 10, None)
    bad = lar.make_items([(1, 0, 0, 0, 10, 0)])
    assert L.lar_sim_streams_workspace(pls, 1, bad, 1, None, 3, ctypes.byref(nb)) == lar.LAR_EINVAL
    rp = (ctypes.c_void_p * 1)(256)
    d = lar.lar_depos(one, one, one, one, one, 10)
    st = (ctypes.c_void_p * 2)(512, 512 + 64)
    # a worker stream equal to the caller's stream, a missing workspace
    assert L.lar_sim_streams(pls, 1, rp, ctypes.byref(d), 3.0, None, its, 1, one, st, 2, one, 1 << 30,
                             ctypes.c_void_p(512)) == lar.LAR_EINVAL
    assert L.lar_sim_streams(pls, 1, rp, ctypes.byref(d), 3.0, None, its, 1, one, st, 2, None, 0,
                             None) == lar.LAR_EWORKSPACE
    d = lar.lar_depos(one, one, one, one, one, 5)     # item reaches past the depos
    assert L.lar_sim_streams(pls, 1, rp, ctypes.byref(d), 3.0, None, its, 1, one, st, 2, one, 1 << 30,
                             None) == lar.LAR_EINVAL


def test_stage_calls_host_side_errors(lar):
    L = lar.lib()
    one = ctypes.c_void_p(256)
    prm = lar.lar_drift_params(1.6, 4e-4, 8.8e-4, 1e4)
    proj = (lar.lar_plane_proj * 9)()
    D = L.lar_drift
    assert D(ctypes.byref(prm), None, None, None, None, None, 0, proj, 3, None, None, None, None, None,
             None) == lar.LAR_OK
    assert D(ctypes.byref(prm), one, one, one, one, one, 5, proj, 9, one, one, one, one, one, None) == lar.LAR_EINVAL
    assert D(ctypes.byref(prm), one, one, one, one, one, 5, proj, 2, one, one, one, one, None,
             None) == lar.LAR_EINVAL
    assert D(ctypes.byref(prm), one, one, one, one, one, -1, proj, 0, one, one, one, one, None,
             None) == lar.LAR_EINVAL
    for bad in ((0.0, 4e-4, 8.8e-4, 0.0), (1.6, -1.0, 8.8e-4, 0.0), (1.6, 4e-4, float("nan"), 0.0)):
        b = lar.lar_drift_params(*bad)
        assert D(ctypes.byref(b), one, one, one, one, one, 5, proj, 0, one, one, one, one, None,
                 None) == lar.LAR_EINVAL
    assert lar.drift_backward_workspace(10) == 2048 * 4 * 8
    B = L.lar_drift_backward
    args = [one] * 11
    assert B(ctypes.byref(prm), one, one, 5, proj, 1, *args, None, 0, None) == lar.LAR_EWORKSPACE
    Z = L.lar_digitize
    assert Z(one, None, 5, 1.0, 0.0, 17, one, None) == lar.LAR_EINVAL
    assert Z(one, None, 5, 1.0, 0.0, 0, one, None) == lar.LAR_EINVAL
    assert Z(one, None, 5, float("inf"), 0.0, 12, one, None) == lar.LAR_EINVAL
    assert Z(None, None, 0, 1.0, 0.0, 12, None, None) == lar.LAR_OK
    P = inputs.cfg1_plane()
    assert lar.noise_workspace(P) == (480 * ((3073 + 15) // 16 * 16) * 8 + 255) // 256 * 256
    pl = lar.make_plane(P)
    assert L.lar_noise(ctypes.byref(pl), one, 0, 0, 300, one, one, 1 << 30, None) == lar.LAR_EINVAL
    assert L.lar_noise(ctypes.byref(pl), one, 0, 0, 1, one, one, 256, None) == lar.LAR_EWORKSPACE


def test_nonfinite_counter_host_side_errors(lar):
    L = lar.lib()
    one = ctypes.c_void_p(16)
    good = lar.lar_depos(one, one, one, one, one, 5)
    assert L.lar_depos_nonfinite(None, one, None) == lar.LAR_EINVAL
    assert L.lar_depos_nonfinite(ctypes.byref(good), None, None) == lar.LAR_EINVAL
    assert L.lar_depos_nonfinite(ctypes.byref(good), ctypes.c_void_p(20), None) == lar.LAR_EINVAL
    for bad in (lar.lar_depos(one, None, one, one, one, 5), lar.lar_depos(one, one, one, one, one, -1)):
        assert L.lar_depos_nonfinite(ctypes.byref(bad), one, None) == lar.LAR_EINVAL
    huge = lar.lar_depos(one, one, one, one, one, 1 << 33)
    assert L.lar_depos_nonfinite(ctypes.byref(huge), one, None) == lar.LAR_ESIZE


def test_atomic_probe_host_side_errors(lar):
    L = lar.lib()
    al = ctypes.c_void_p(256)
    assert L.lar_atomic_probe(None, 64, 1, None) == lar.LAR_EINVAL
    assert L.lar_atomic_probe(ctypes.c_void_p(260), 64, 1, None) == lar.LAR_EINVAL
    assert L.lar_atomic_probe(al, 63, 1, None) == lar.LAR_EINVAL
    assert L.lar_atomic_probe(al, 64, -1, None) == lar.LAR_EINVAL


def test_philox_probe_host_side_errors(lar):
    L = lar.lib()
    a = ctypes.c_void_p(256)
    assert L.lar_philox_probe(None, 256, 10, None) == lar.LAR_EINVAL
    assert L.lar_philox_probe(ctypes.c_void_p(260), 256, 10, None) == lar.LAR_EINVAL
    for n_threads in (0, 255, 257, -256):
        assert L.lar_philox_probe(a, n_threads, 10, None) == lar.LAR_EINVAL
    assert L.lar_philox_probe(a, 256, -1, None) == lar.LAR_EINVAL


def test_row_copy_probe_host_side_errors(lar):
    L = lar.lib()
    a = ctypes.c_void_p(256)
    ok = (a, 6000, 6000, 4, a, 3088, 3073, 2, None)
    assert L.lar_row_copy_probe(a, 6000, 6000, 0, None, 0, 0, 2, None) == lar.LAR_OK   # nothing to copy
    for i, bad in ((0, None), (1, 5999), (2, 6001), (2, 6146), (3, -1), (4, None), (5, 3000), (6, 3074), (6, 0),
                   (7, 0), (7, 17), (0, ctypes.c_void_p(260)), (4, ctypes.c_void_p(260))):
        args = list(ok)
        args[i] = bad
        assert L.lar_row_copy_probe(*args) == lar.LAR_EINVAL, (i, bad)


def test_schedule_registry_host_side(lar):
    P = inputs.cfg1_plane()
    d = lar.schedule_default(P)
    assert d == dict(row_threads=384, row_order=4, wire_cols=16, wire_threads=1024, wire_order=0, raster_tile=512)
    assert lar.schedule_get(P) == d
    cands = lar.schedule_candidates(P)
    assert cands[0] == d and len(cands) == len({tuple(c.values()) for c in cands})
    other = dict(d, wire_cols=16, wire_threads=1024, wire_order=1, row_threads=1024, raster_tile=640)
    lar.schedule_set(P, other)
    try:
        assert lar.schedule_get(P) == other
        Q = inputs.cfg1_plane()
        Q.n_wires = 470                     # another shape keeps the built-in schedule
        assert lar.schedule_get(Q) == lar.schedule_default(Q)
    finally:
        lar.schedule_set(P, None)
    assert lar.schedule_get(P) == d
    # Tf/2 = 3072 over 256 threads is 12 values per thread; 4 x 1024 is not a
    # wire shape; radix order 5 needs 36 | n (3072 is not), order 6 does not
    # exist; 16 x 512 is 16 values of Wf 512; 4 x 576 needs Wf 864's order 5
    for bad in (dict(row_threads=256), dict(wire_cols=4, wire_threads=1024), dict(row_order=5),
                dict(row_order=6), dict(wire_cols=4, wire_threads=576),
                dict(wire_order=-1), dict(wire_cols=16, wire_threads=512), dict(row_threads=300),
                dict(raster_tile=500), dict(raster_tile=1024)):
        with pytest.raises(lar.LarError) as e:
            lar.schedule_set(P, dict(d, **bad))
        assert e.value.status == lar.LAR_EINVAL
    assert lar.schedule_get(P) == d
    Q = inputs.cfg1_plane()
    Q.nw_fft = 500                          # no 2^a 3^b plan
    with pytest.raises(lar.LarError) as e:
        lar.schedule_default(Q)
    assert e.value.status == lar.LAR_ESIZE


def test_schedule_candidates_every_shape_valid(lar):
    # every listed candidate is accepted by lar_schedule_set, for small and
    # large transforms; the power-of-8 wire length lists one radix order
    for P in (inputs.cfg0_plane(), inputs.cfg1_plane(), inputs.Plane(n_wires=800, n_ticks=6000),
              inputs.Plane(n_wires=3, n_ticks=2, n_imp=1, nt_fft=2, nw_fft=3),
              inputs.Plane(n_wires=10, n_ticks=16000, n_imp=2, nt_fft=16384, nw_fft=16)):
        cands = lar.schedule_candidates(P)
        assert cands
        try:
            for c in cands:
                lar.schedule_set(P, c)
                assert lar.schedule_get(P) == c
        finally:
            lar.schedule_set(P, None)
    wire_orders = {c["wire_order"] for c in lar.schedule_candidates(inputs.cfg1_plane())}
    assert wire_orders == {0, 1}            # 512 = 8^3: orders 2, 3 and 4 repeat order 0
    row_orders = {c["row_order"] for c in lar.schedule_candidates(inputs.cfg1_plane())}
    assert 4 in row_orders                  # 3072 = 8 8 8 6 with a radix-6 pass
    tiles = {c["raster_tile"] for c in lar.schedule_candidates(inputs.cfg1_plane())}
    assert tiles == {384, 512, 640, 768}
    # the 800-wire planes (Wf 864) default to the compile-time 6 4 6 6 wire pass
    U = inputs.Plane(n_wires=800, n_ticks=6000, kind="bipolar")
    d = lar.schedule_default(U)
    assert (U.nw_fft, d["wire_cols"], d["wire_threads"], d["wire_order"]) == (864, 4, 576, 5)
    assert any(c["wire_order"] == 0 and c["wire_threads"] == 512 for c in lar.schedule_candidates(U))
