"""Launch schedules of the FFT convolution: every candidate schedule the
library lists gives the oracle's waveforms (relative L2 1e-5), the
autotuner registers a listed schedule, and a batch plan built under a
non-default schedule still equals the single-plane calls."""
import numpy as np
import pytest

import oracle
from paper_2203_02479_amd import inputs

pytestmark = pytest.mark.gpu

RTOL_L2 = 1e-5


def rel_l2(a, b):
    cplx = np.iscomplexobj(a) or np.iscomplexobj(b)    # complex arrays keep their imaginary part
    a = np.asarray(a, np.complex128 if cplx else np.float64)
    b = np.asarray(b, np.complex128 if cplx else np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


SHAPES = [
    dict(n_wires=64, n_ticks=1024, n_imp=10, nt_fft=1024, nw_fft=96),    # tiny plane shape
    dict(n_wires=30, n_ticks=1000, n_imp=10, nt_fft=1024, nw_fft=864),   # ragged column tiles
    dict(n_wires=21, n_ticks=6000, n_imp=4, nt_fft=6144, nw_fft=512),
    dict(n_wires=7, n_ticks=100, n_imp=3, nt_fft=108, nw_fft=12),
]


@pytest.mark.parametrize("case", SHAPES)
def test_every_candidate_schedule_matches_oracle(case):
    import torch
    from paper_2203_02479_amd import lar
    P = inputs.Plane(**case)
    g = inputs.random_grid(P, 31, density=0.3)
    R = inputs.random_spectrum(P, 32)
    ref = oracle.conv_fft(P, g, R)
    gd = torch.as_tensor(g, dtype=torch.float32).cuda().contiguous()
    rd = torch.as_tensor(R, dtype=torch.float32).cuda().contiguous()
    wave = torch.empty((P.n_wires, P.n_ticks), dtype=torch.float32, device="cuda")
    ws = lar.workspace(lar.fftconv_workspace(P))
    cands = lar.schedule_candidates(P)
    assert cands
    try:
        for c in cands:
            print(f"schedule {c}", flush=True)
            lar.schedule_set(P, c)
            wave.fill_(float("nan"))
            lar.fftconv(P, gd, rd, wave, ws)
            torch.cuda.synchronize()
            w = wave.cpu().numpy()
            assert np.isfinite(w).all(), c
            assert rel_l2(w, ref) < RTOL_L2, c
            assert np.max(np.abs(w - ref)) <= RTOL_L2 * np.max(np.abs(ref)), c
    finally:
        lar.schedule_set(P, None)


def test_autotune_registers_a_listed_schedule(tmp_path, monkeypatch):
    from paper_2203_02479_amd import autotune, lar
    monkeypatch.setenv("LAR_TUNE_CACHE", str(tmp_path / "sched.json"))
    P = inputs.Plane(**SHAPES[0])
    try:
        out = autotune.tune(P, reps=3, warmup=1)
        assert out["schedule"] == lar.schedule_get(P)
        listed = lar.schedule_candidates(P)
        rows = {(c["row_threads"], c["row_order"]) for c in listed}
        wires = {(c["wire_cols"], c["wire_threads"], c["wire_order"]) for c in listed}
        s = out["schedule"]
        assert (s["row_threads"], s["row_order"]) in rows
        assert (s["wire_cols"], s["wire_threads"], s["wire_order"]) in wires
        lar.schedule_set(P, None)
        assert autotune.load([P]) == 1
        assert lar.schedule_get(P) == s
    finally:
        lar.schedule_set(P, None)


def test_batch_under_non_default_schedule():
    import torch
    from paper_2203_02479_amd import lar
    planes = [inputs.Plane(n_wires=40, n_ticks=700, kind="bipolar")]
    P = planes[0]
    resps = [lar.spectrum_from_time(P, inputs.response_time(P.n_imp, P.half_w, 200, P.kind))]
    d = lar.schedule_default(P)
    alt = dict(d, wire_cols=4, wire_threads=256, row_threads=1024, row_order=1, raster_tile=384)
    deps = [inputs.random_depos(P, n, seed=300 + i, margin=0.1) for i, n in enumerate((900, 0, 2500))]
    items, off, woff = [], 0, 0
    for i, dep in enumerate(deps):
        items.append((0, i, 0, off, len(dep), woff))
        off += len(dep)
        woff += P.n_wires * P.n_ticks
    cat = inputs.Depos(*(np.concatenate([x.arrays()[k] for x in deps]) for k in range(5)))
    try:
        lar.schedule_set(P, alt)
        D = lar.DeviceDepos.from_host(cat)
        wave = torch.zeros(woff, device="cuda")
        ws = lar.workspace(lar.batch_workspace(planes, items, None))
        b = lar.Batch(planes, resps, D, 3.0, None, items, wave, ws, use_graph=True)
        for rep in range(2):
            wave.fill_(-1.0)
            b.run()
            torch.cuda.synchronize()
            got = wave.cpu().numpy()
            for (pt, e, pl, o, n, wo), dep in zip(items, deps):
                Dd = lar.DeviceDepos.from_host(dep)
                w = torch.empty((P.n_wires, P.n_ticks), device="cuda")
                lar.sim_plane(P, Dd, 3.0, None, resps[0], w, lar.workspace(lar.sim_plane_workspace(P, n)))
                torch.cuda.synchronize()
                ref = w.cpu().numpy().reshape(-1)
                assert rel_l2(got[wo:wo + ref.size], ref) < RTOL_L2
        b.close()
    finally:
        lar.schedule_set(P, None)


def test_every_raster_tile_matches_oracle(tmp_path, monkeypatch):
    """Each listed raster tile: the mean grid within the oracle's tolerance,
    the binomial grid nearly equal to the oracle's and identical bit for bit
    across tiles (whether a sub-chunk sums in the tile or adds straight to
    the grid changes no count); tune_raster registers a listed tile."""
    import torch
    from paper_2203_02479_amd import autotune, lar
    monkeypatch.setenv("LAR_TUNE_CACHE", str(tmp_path / "sched.json"))
    ev = inputs.cfg0_event()
    P, dep = ev.planes[0], ev.depos[0]
    dep.sigma_t[::7] *= 2.5          # wider bounding boxes: some sub-chunks exceed the small tiles
    D = lar.DeviceDepos.from_host(dep)
    ref_mean = oracle.raster_mean(P, dep, inputs.NSIGMA)
    fl = (1, 99, 3, 1)
    ref_fl = oracle.raster_fluct(P, dep, inputs.NSIGMA, mode=1, seed=99, event=3, plane_id=1)
    grid = torch.zeros((P.n_rows, P.n_ticks), dtype=torch.float32, device="cuda")
    tiles = sorted({c["raster_tile"] for c in lar.schedule_candidates(P)})
    assert tiles == [384, 512, 640, 768]
    first = None
    try:
        for tile in tiles:
            print(f"raster tile {tile}", flush=True)
            lar.schedule_set(P, dict(lar.schedule_default(P), raster_tile=tile))
            grid.zero_()
            lar.raster(P, D, inputs.NSIGMA, None, grid, None)
            torch.cuda.synchronize()
            g = grid.cpu().numpy()
            assert rel_l2(g, ref_mean) < RTOL_L2, tile
            assert np.max(np.abs(g - ref_mean)) <= 1e-5 * np.max(np.abs(ref_mean)), tile
            grid.zero_()
            lar.raster(P, D, inputs.NSIGMA, fl, grid, lar.workspace(lar.raster_workspace(P, len(dep), fl)))
            torch.cuda.synchronize()
            g = grid.cpu().numpy()
            assert np.mean(g == ref_fl) > 0.9999, tile
            if first is None:
                first = g
            assert np.array_equal(g, first), tile
        lar.schedule_set(P, None)
        out = autotune.tune_raster(P, D, inputs.NSIGMA, fl, reps=2, warmup=1)
        assert out["raster_tile"] in tiles and set(out["ms"]) == set(tiles)
        assert lar.schedule_get(P)["raster_tile"] == out["raster_tile"]
    finally:
        lar.schedule_set(P, None)
