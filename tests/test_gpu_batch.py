"""Batched plan (items per plane type in waves: one raster launch and one
launch per FFT stage per wave, hipGraph replay) against per-item
lar_sim_plane runs and against the FP64 oracle at the three-plane geometry
(800-wire bipolar induction planes, Wf 864, and the 480-wire collection
plane, 6000 ticks); the batched backward against the oracle's gradients
summed over items."""
import numpy as np
import pytest

import oracle
from paper_2203_02479_amd import inputs

pytestmark = pytest.mark.gpu


def _setup(n_events=3, fluct_mode=1, sizes=None, seed=7, widen=False):
    import torch
    from paper_2203_02479_amd import lar
    planes = [inputs.Plane(n_wires=40, n_ticks=700, kind="bipolar"),
              inputs.Plane(n_wires=24, n_ticks=700, kind="unipolar")]
    resps = [lar.spectrum_from_time(p, inputs.response_time(p.n_imp, p.half_w, 200, p.kind)) for p in planes]
    rng = np.random.default_rng(seed)
    items, deps, off, woff = [], [], 0, 0
    for e in range(n_events):
        for pl, pt in ((0, 0), (1, 0), (2, 1)):
            n = int(rng.integers(0, 3000)) if sizes is None else sizes[(e * 3 + pl) % len(sizes)]
            d = inputs.random_depos(planes[pt], n, seed=seed * 100 + e * 3 + pl, margin=0.1)
            if widen:   # windows beyond the raster kernel's 16 x 32 weight slots
                d.sigma_t[::5] *= 4.0
                d.sigma_x[2::5] *= 3.0
            items.append((pt, e, pl, off, n, woff))
            deps.append(d)
            off += n
            woff += planes[pt].n_wires * planes[pt].n_ticks + 2
    cat = inputs.Depos(*(np.concatenate([d.arrays()[k] for d in deps]) if deps else np.zeros(0, np.float32)
                         for k in range(5)))
    fl = (fluct_mode, 4242, 0, 0) if fluct_mode else None
    return torch, lar, planes, resps, items, deps, cat, fl, woff


def _reference(torch, lar, planes, resps, items, deps, fl, total):
    ref = torch.zeros(total, device="cuda")
    for (pt, e, pl, off, n, wo), d in zip(items, deps):
        P = planes[pt]
        D = lar.DeviceDepos.from_host(d)
        f = (fl[0], fl[1], e, pl) if fl else None
        ws = lar.workspace(lar.sim_plane_workspace(P, n, f))
        w = torch.empty((P.n_wires, P.n_ticks), device="cuda")
        lar.sim_plane(P, D, 3.0, f, resps[pt], w, ws)
        ref[wo:wo + w.numel()] = w.reshape(-1)
    torch.cuda.synchronize()
    return ref.cpu().numpy()


@pytest.mark.parametrize("mode,use_graph,max_wave", [(1, True, 0), (1, False, 0), (2, True, 0), (0, True, 0),
                                                    (1, True, 1), (3, True, 2), (0, True, 2)])
def test_batch_matches_single_plane_runs(mode, use_graph, max_wave):
    torch, lar, planes, resps, items, deps, cat, fl, total = _setup(fluct_mode=mode)
    D = lar.DeviceDepos.from_host(cat)
    wave = torch.full((total,), -7.0, device="cuda")
    ws = lar.workspace(lar.batch_workspace(planes, items, fl, max_wave=max_wave))
    b = lar.Batch(planes, resps, D, 3.0, fl, items, wave, ws, use_graph=use_graph)
    n_waves, largest = b.waves()
    # 3 events: 6 items of type 0, 3 of type 1
    assert largest == (6 if max_wave == 0 else max_wave)
    assert n_waves == (2 if max_wave == 0 else -(-6 // max_wave) - (-3 // max_wave))
    ref = _reference(torch, lar, planes, resps, items, deps, fl, total)
    for rep in range(3):
        wave.fill_(-7.0)                 # eager work between replays
        b.run()
        torch.cuda.synchronize()
        got = wave.cpu().numpy()
        gaps = np.ones(total, bool)
        for (pt, e, pl, off, n, wo) in items:
            gaps[wo:wo + planes[pt].n_wires * planes[pt].n_ticks] = False
        assert np.all(got[gaps] == -7.0)    # untouched between items
        if mode:
            assert np.array_equal(got[~gaps], ref[~gaps]), rep
        else:
            np.testing.assert_allclose(got[~gaps], ref[~gaps], rtol=0, atol=1e-5 * np.abs(ref).max())
    b.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_runs_back_to_back(use_graph):
    """Runs queued without a synchronisation between them: the FFT stages of
    one run's last waves (on the plan's second stream) finish before the next
    run clears the grid regions, so the last run's waveforms are exact."""
    torch, lar, planes, resps, items, deps, cat, fl, total = _setup(fluct_mode=1)
    D = lar.DeviceDepos.from_host(cat)
    wave = torch.full((total,), -7.0, device="cuda")
    ws = lar.workspace(lar.batch_workspace(planes, items, fl, max_wave=1))
    b = lar.Batch(planes, resps, D, 3.0, fl, items, wave, ws, use_graph=use_graph)
    assert b.waves()[0] == 9
    ref = _reference(torch, lar, planes, resps, items, deps, fl, total)
    for _ in range(4):
        b.run()
    torch.cuda.synchronize()
    got = wave.cpu().numpy()
    for (pt, e, pl, off, n, wo) in items:
        sl = slice(wo, wo + planes[pt].n_wires * planes[pt].n_ticks)
        assert np.array_equal(got[sl], ref[sl]), (e, pl)
    b.close()


def test_batch_waves_of_unequal_size():
    """Waves of unequal size and plane type (7 items of the larger type in
    waves of 3, 3, 1, then 6 of the smaller in waves of 3, 3), so that a
    wave's grids are larger than an earlier, smaller wave's: each wave's
    grids, spectra and outputs keep regions of their own while the FFT
    stages of earlier waves still run, and the waveforms match per-item
    runs exactly."""
    import torch
    from paper_2203_02479_amd import lar
    planes = [inputs.Plane(n_wires=40, n_ticks=700, kind="bipolar"),
              inputs.Plane(n_wires=24, n_ticks=700, kind="unipolar")]
    resps = [lar.spectrum_from_time(p, inputs.response_time(p.n_imp, p.half_w, 200, p.kind)) for p in planes]
    items, deps, off, woff = [], [], 0, 0
    for i, pt in enumerate([0] * 7 + [1] * 6):
        d = inputs.random_depos(planes[pt], 1200 + 97 * i, seed=900 + i, margin=0.1)
        items.append((pt, i, pt, off, len(d.q), woff))
        deps.append(d)
        off += len(d.q)
        woff += planes[pt].n_wires * planes[pt].n_ticks
    cat = inputs.Depos(*(np.concatenate([d.arrays()[k] for d in deps]) for k in range(5)))
    fl = (1, 4242, 0, 0)
    ref = _reference(torch, lar, planes, resps, items, deps, fl, woff)
    D = lar.DeviceDepos.from_host(cat)
    for use_graph in (True, False):
        wave = torch.full((woff,), -7.0, device="cuda")
        ws = lar.workspace(lar.batch_workspace(planes, items, fl, max_wave=3))
        b = lar.Batch(planes, resps, D, 3.0, fl, items, wave, ws, use_graph=use_graph)
        assert b.waves() == (5, 3)
        for _ in range(3):
            b.run()
        torch.cuda.synchronize()
        assert np.array_equal(wave.cpu().numpy(), ref), use_graph
        b.close()


def test_batch_single_wave():
    """One plane type in one wave (one grid region, the FFT stages still on
    the plan's second stream): exact waveforms, graph and eager, run twice."""
    import torch
    from paper_2203_02479_amd import lar
    planes = [inputs.Plane(n_wires=24, n_ticks=700, kind="unipolar")]
    resps = [lar.spectrum_from_time(planes[0], inputs.response_time(planes[0].n_imp, planes[0].half_w, 200,
                                                                    planes[0].kind))]
    items, deps, off, woff = [], [], 0, 0
    for i in range(4):
        d = inputs.random_depos(planes[0], 900 + 50 * i, seed=700 + i, margin=0.1)
        items.append((0, i, 2, off, len(d.q), woff))
        deps.append(d)
        off += len(d.q)
        woff += planes[0].n_wires * planes[0].n_ticks
    cat = inputs.Depos(*(np.concatenate([d.arrays()[k] for d in deps]) for k in range(5)))
    fl = (1, 99, 0, 0)
    ref = _reference(torch, lar, planes, resps, items, deps, fl, woff)
    D = lar.DeviceDepos.from_host(cat)
    for use_graph in (True, False):
        wave = torch.full((woff,), -7.0, device="cuda")
        ws = lar.workspace(lar.batch_workspace(planes, items, fl))
        b = lar.Batch(planes, resps, D, 3.0, fl, items, wave, ws, use_graph=use_graph)
        assert b.waves() == (1, 4)
        b.run()
        b.run()
        torch.cuda.synchronize()
        assert np.array_equal(wave.cpu().numpy(), ref), use_graph
        b.close()


def test_batch_with_empty_items_and_one_item():
    torch, lar, planes, resps, items, deps, cat, fl, total = _setup(n_events=2, sizes=[0, 1500, 0, 700, 0, 0])
    D = lar.DeviceDepos.from_host(cat)
    wave = torch.zeros(total, device="cuda")
    ws = lar.workspace(lar.batch_workspace(planes, items, fl))
    b = lar.Batch(planes, resps, D, 3.0, fl, items, wave, ws)
    b.run()
    torch.cuda.synchronize()
    ref = _reference(torch, lar, planes, resps, items, deps, fl, total)
    assert np.array_equal(wave.cpu().numpy(), ref)
    b.close()


@pytest.mark.parametrize("mode", [1, 0])
def test_batch_with_wide_depos(mode):
    """Depos wider than the hot raster kernel's weight slots, taken by the
    flagged-sub-chunk kernel (fluctuated) or the wide-depo kernel (mean)
    through the batch's item table: the same waveforms as per-item runs."""
    torch, lar, planes, resps, items, deps, cat, fl, total = _setup(n_events=2, fluct_mode=mode, widen=True)
    D = lar.DeviceDepos.from_host(cat)
    wave = torch.zeros(total, device="cuda")
    ws = lar.workspace(lar.batch_workspace(planes, items, fl))
    b = lar.Batch(planes, resps, D, 3.0, fl, items, wave, ws)
    b.run()
    torch.cuda.synchronize()
    ref = _reference(torch, lar, planes, resps, items, deps, fl, total)
    got = wave.cpu().numpy()
    if mode:
        assert np.array_equal(got, ref)
    else:
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-5 * np.abs(ref).max())
    b.close()


# ------------------------------------------------------------------ oracle parity at full geometry

def rel_l2(a, b):
    cplx = np.iscomplexobj(a) or np.iscomplexobj(b)    # complex arrays keep their imaginary part
    a = np.asarray(a, np.complex128 if cplx else np.float64)
    b = np.asarray(b, np.complex128 if cplx else np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _three_plane_batch(n_events, n_track, n_points, seed0):
    """Events of the three-plane geometry (U, V: 800 wires, bipolar, Wf 864;
    W: 480 wires, unipolar; 6000 ticks) as batch items of two plane types."""
    import torch
    from paper_2203_02479_amd import lar
    evs = [inputs.cfg2_event(seed=seed0 + e, n_track=n_track, n_points=n_points, n_seg=max(1, n_track // 8333))
           for e in range(n_events)]
    planes = [evs[0].planes[0], evs[0].planes[2]]
    rtime = [inputs.response_time(p.n_imp, p.half_w, inputs.RESP_TICKS, p.kind) for p in planes]
    resps = [lar.spectrum_from_time(p, r) for p, r in zip(planes, rtime)]
    items, chunks, off, woff = [], [], 0, 0
    for e, ev in enumerate(evs):
        for pl in range(3):
            pt = 0 if pl < 2 else 1
            d = ev.depos[pl]
            items.append((pt, e, pl, off, len(d), woff))
            chunks.append(d)
            off += len(d)
            woff += planes[pt].n_wires * planes[pt].n_ticks
    cat = inputs.Depos(*(np.concatenate([c.arrays()[k] for c in chunks]) for k in range(5)))
    return torch, lar, planes, rtime, resps, items, chunks, cat, woff


@pytest.mark.parametrize("mode,max_wave", [(0, 0), (1, 2)])
def test_batch_three_planes_vs_oracle(mode, max_wave):
    """Each item's waveforms against the oracle: the mean path within
    relative L2 1e-5 and max |diff| 1e-5 of max |ref|; fluctuated items
    against the oracle's convolution of its fluctuated grid under the same
    keys (nearly every bin identical: relative L2 1e-4)."""
    torch, lar, planes, rtime, resps, items, chunks, cat, total = _three_plane_batch(2, 40_000, 2_000,
                                                                                    inputs.SEED0 + 600)
    fl = (mode, 555, 0, 0) if mode else None
    D = lar.DeviceDepos.from_host(cat)
    wave = torch.full((total,), float("nan"), device="cuda")
    ws = lar.workspace(lar.batch_workspace(planes, items, fl, max_wave=max_wave))
    b = lar.Batch(planes, resps, D, inputs.NSIGMA, fl, items, wave, ws)
    b.run()
    torch.cuda.synchronize()
    got_all = wave.cpu().numpy()
    b.close()
    Rc = [oracle.response_spectrum(p, r) for p, r in zip(planes, rtime)]
    for (pt, e, pl, off, n, wo), d in zip(items, chunks):
        P = planes[pt]
        got = got_all[wo:wo + P.n_wires * P.n_ticks].reshape(P.n_wires, P.n_ticks)
        if mode == 0:
            ref = oracle.sim_plane_mean(P, d, Rc[pt])
            assert rel_l2(got, ref) < 1e-5, (e, pl)
            assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)), (e, pl)
        else:
            S = oracle.raster_fluct(P, d, inputs.NSIGMA, mode=mode, seed=555, event=e, plane_id=pl)
            ref = oracle.conv_fft(P, S, Rc[pt])
            assert rel_l2(got, ref) < 1e-4, (e, pl)


def test_full_three_plane_event_vs_oracle():
    """One full event of the three-plane configuration (1.9M track depos and
    100k point depos with q log-uniform in 1e2..1e5) through lar_sim_plane
    per plane: mean waveforms within relative L2 1e-5 and max |diff| 1e-5 of
    max |ref|; binomial grids with at least 99.99% of the non-zero bins equal
    to the oracle's."""
    import torch
    from paper_2203_02479_amd import lar
    ev = inputs.cfg2_event()
    for pl in range(3):
        P, dep = ev.planes[pl], ev.depos[pl]
        r = inputs.response_time(P.n_imp, P.half_w, inputs.RESP_TICKS, P.kind)
        D = lar.DeviceDepos.from_host(dep)
        resp = lar.spectrum_from_time(P, r)
        wave = torch.empty((P.n_wires, P.n_ticks), device="cuda")
        lar.sim_plane(P, D, inputs.NSIGMA, None, resp, wave, lar.workspace(lar.sim_plane_workspace(P)))
        torch.cuda.synchronize()
        got = wave.cpu().numpy()
        ref = oracle.sim_plane_mean(P, dep, oracle.response_spectrum(P, r))
        assert rel_l2(got, ref) < 1e-5, pl
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)), pl
        del wave
        fl = (1, inputs.SEED0 + 200, 0, pl)
        grid = torch.zeros((P.n_rows, P.n_ticks), device="cuda")
        lar.raster(P, D, inputs.NSIGMA, fl, grid, lar.workspace(lar.raster_workspace(P, len(dep), fl)))
        torch.cuda.synchronize()
        g = grid.cpu().numpy()
        del grid
        S = oracle.raster_fluct(P, dep, inputs.NSIGMA, mode=1, seed=inputs.SEED0 + 200, event=0, plane_id=pl)
        nz = (g != 0) | (S != 0)
        assert np.mean(g[nz] == S[nz]) > 0.9999, pl
        assert abs(g.sum() - S.sum()) < 1e-4 * abs(S.sum())


def test_batch_backward_vs_oracle():
    """The batched backward (waves of 2 items, so the response gradient
    accumulates across waves) against the oracle: grid-path gradients per
    item (conv_adjoint then raster_adjoint) and the response gradient summed
    over the items of each plane type, relative L2 1e-4 each."""
    torch, lar, planes, rtime, resps, items, chunks, cat, total = _three_plane_batch(2, 20_000, 1_000,
                                                                                    inputs.SEED0 + 700)
    # one item without depos
    pt, e, pl, off, n, wo = items[1]
    items[1] = (pt, e, pl, off, 0, wo)
    D = lar.DeviceDepos.from_host(cat)
    wave = torch.empty(total, device="cuda")
    ws = lar.workspace(lar.batch_workspace(planes, items, None, max_wave=2))
    b = lar.Batch(planes, resps, D, inputs.NSIGMA, None, items, wave, ws)
    assert b.waves() == (3, 2)
    G = np.random.default_rng(5).standard_normal(total).astype(np.float32)
    Gd = torch.as_tensor(G).cuda()
    runs = []
    # without a forward run every wave is recomputed; right after a run the
    # last wave's spectra are reused
    for with_run in (False, True):
        rg = [torch.full_like(r, float("nan")) for r in resps]
        dg = [torch.full((len(cat),), float("nan"), device="cuda") for _ in range(5)]
        if with_run:
            b.run()
        b.backward(Gd, rg, dg)
        torch.cuda.synchronize()
        runs.append(([r.cpu().numpy().astype(np.float64) for r in rg], [d.cpu().numpy() for d in dg]))
    b.close()
    Rc = [oracle.response_spectrum(p, r) for p, r in zip(planes, rtime)]
    dR_ref = [np.zeros_like(R) for R in Rc]
    for (pt, e, pl, off, n, wo), d in zip(items, chunks):
        P = planes[pt]
        d = d.take(slice(0, n))
        S = oracle.raster_mean(P, d, inputs.NSIGMA)
        Gi = G[wo:wo + P.n_wires * P.n_ticks].reshape(P.n_wires, P.n_ticks).astype(np.float64)
        GS, dR = oracle.conv_adjoint(P, S, Rc[pt], Gi)
        dR_ref[pt] += dR
        if n == 0:
            continue
        ref = oracle.raster_adjoint(P, d, inputs.NSIGMA, GS)
        for rg_np, dg_np in runs:
            for k, name in enumerate(("q", "t", "x", "sigma_t", "sigma_x")):
                assert rel_l2(dg_np[k][off:off + n], ref[k]) < 1e-4, (e, pl, name)
    for rg_np, _ in runs:
        for t in range(2):
            got = rg_np[t]
            assert rel_l2(got[..., 0] + 1j * got[..., 1], dR_ref[t]) < 1e-4, t


# ------------------------------------------------------------------ concurrent streams

@pytest.mark.parametrize("mode,n_streams", [(1, 3), (0, 2), (3, 4), (1, 1)])
def test_streams_match_single_plane_runs(mode, n_streams):
    """Items spread over several streams give the per-item lar_sim_plane
    waveforms (fluctuated counts exactly), ordered after earlier work on the
    caller's stream and before later work."""
    torch, lar, planes, resps, items, deps, cat, fl, total = _setup(fluct_mode=mode)
    D = lar.DeviceDepos.from_host(cat)
    ref = _reference(torch, lar, planes, resps, items, deps, fl, total)
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    ws = lar.workspace(lar.sim_streams_workspace(planes, items, fl, n_streams))
    wave = torch.empty(total, device="cuda")
    for rep in range(3):
        wave.fill_(-7.0)                              # earlier work on the caller's stream
        lar.sim_streams(planes, resps, D, 3.0, fl, items, wave, streams, ws)
        snap = wave.clone()                           # later work on the caller's stream
        torch.cuda.synchronize()
        got = snap.cpu().numpy()
        gaps = np.ones(total, bool)
        for (pt, e, pl, off, n, wo) in items:
            gaps[wo:wo + planes[pt].n_wires * planes[pt].n_ticks] = False
        assert np.all(got[gaps] == -7.0)
        if mode:
            assert np.array_equal(got[~gaps], ref[~gaps]), rep
        else:
            np.testing.assert_allclose(got[~gaps], ref[~gaps], rtol=0, atol=1e-5 * np.abs(ref).max())


def test_streams_three_planes_vs_oracle():
    """Two events of the three-plane geometry on four streams, mean path:
    each item against the oracle (relative L2 1e-5, max |diff| 1e-5 of max
    |ref|)."""
    torch, lar, planes, rtime, resps, items, chunks, cat, total = _three_plane_batch(2, 30_000, 1_500,
                                                                                    inputs.SEED0 + 800)
    D = lar.DeviceDepos.from_host(cat)
    streams = [torch.cuda.Stream() for _ in range(4)]
    ws = lar.workspace(lar.sim_streams_workspace(planes, items, None, 4))
    wave = torch.full((total,), float("nan"), device="cuda")
    lar.sim_streams(planes, resps, D, inputs.NSIGMA, None, items, wave, streams, ws)
    torch.cuda.synchronize()
    got_all = wave.cpu().numpy()
    Rc = [oracle.response_spectrum(p, r) for p, r in zip(planes, rtime)]
    for (pt, e, pl, off, n, wo), d in zip(items, chunks):
        P = planes[pt]
        got = got_all[wo:wo + P.n_wires * P.n_ticks].reshape(P.n_wires, P.n_ticks)
        ref = oracle.sim_plane_mean(P, d, Rc[pt])
        assert rel_l2(got, ref) < 1e-5, (e, pl)
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)), (e, pl)
