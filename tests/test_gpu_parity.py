"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded float32 inputs.  Tolerances: waveforms and grids within relative
L2 1e-5 (mean path); fluctuated counts bit-exact on injected (q, p, counter)
triples; fluctuated grids by identity of (almost) every bin and by
chi-square on mean and variance."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_02479_amd import inputs

pytestmark = pytest.mark.gpu

RTOL_L2 = 1e-5


def _lar():
    from paper_2203_02479_amd import lar
    return lar


def _torch():
    import torch
    return torch


def rel_l2(a, b):
    cplx = np.iscomplexobj(a) or np.iscomplexobj(b)    # complex arrays keep their imaginary part
    a = np.asarray(a, np.complex128 if cplx else np.float64)
    b = np.asarray(b, np.complex128 if cplx else np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def gpu_raster(plane, dep, nsigma=3.0, fluct=None, ws_bytes=None):
    torch, lar = _torch(), _lar()
    D = lar.DeviceDepos.from_host(dep)
    grid = torch.zeros((plane.n_rows, plane.n_ticks), dtype=torch.float32, device="cuda")
    nb = lar.raster_workspace(plane, len(dep), fluct) if ws_bytes is None else ws_bytes
    ws = lar.workspace(nb) if nb else None
    lar.raster(plane, D, nsigma, fluct, grid, ws)
    torch.cuda.synchronize()
    return grid.cpu().numpy()


def gpu_fftconv(plane, grid_np, resp_np):
    torch, lar = _torch(), _lar()
    g = torch.as_tensor(grid_np, dtype=torch.float32).cuda().contiguous()
    r = torch.as_tensor(resp_np, dtype=torch.float32).cuda().contiguous()
    wave = torch.full((plane.n_wires, plane.n_ticks), float("nan"), dtype=torch.float32, device="cuda")
    ws = lar.workspace(lar.fftconv_workspace(plane))
    lar.fftconv(plane, g, r, wave, ws)
    torch.cuda.synchronize()
    return wave.cpu().numpy()


# ------------------------------------------------------------------ raster

def test_raster_mean_cfg0():
    ev = inputs.cfg0_event()
    P, dep = ev.planes[0], ev.depos[0]
    g = gpu_raster(P, dep)
    ref = oracle.raster_mean(P, dep)
    assert rel_l2(g, ref) < RTOL_L2
    assert np.abs(g - ref).max() < 1e-5 * np.abs(ref).max()
    assert g.sum() == pytest.approx(ref.sum(), rel=1e-6)


@pytest.mark.parametrize("n,seed,sig,margin", [(1, 1, 1.0, 0.0), (127, 2, 1.0, 0.3), (129, 3, 1.0, 0.3),
                                               (1000, 4, 1.0, 0.2), (3000, 5, 6.0, 0.1),
                                               (500, 6, 40.0, 0.5)])
def test_raster_random_depos_edges(n, seed, sig, margin):
    """Ragged chunk counts, clipping at every border, windows beyond the
    per-depo slots (sigma x6, x40) and scattered (non-track) order."""
    P = inputs.Plane(n_wires=20, n_ticks=300, n_imp=10)
    dep = inputs.random_depos(P, n, seed, sigma_scale=sig, margin=margin)
    g = gpu_raster(P, dep)
    ref = oracle.raster_mean(P, dep)
    assert rel_l2(g, ref) < RTOL_L2


def test_raster_degenerate_depos():
    P = inputs.Plane(n_wires=8, n_ticks=64, n_imp=4)
    f = np.float32
    q = f([100, -50, 7, 3, 5, 9, 11, 13])
    t = f([10.0, 12.3, np.nan, 5.0, -100.0, 8.0, 31.999, 0.0])
    x = f([7.0, 11.1, 3.0, np.inf, 5.0, 19.99, 0.0, 39.999])
    st = f([0.0, 0.7, 0.5, 0.5, 0.5, -1.0, 1e-9, 0.3])
    sx = f([0.0, 0.9, 0.5, 0.5, 0.5, 0.8, 2.0, 0.0])
    dep = inputs.Depos(q, t, x, st, sx)
    g = gpu_raster(P, dep)
    ref = oracle.raster_mean(P, dep)
    assert rel_l2(g, ref) < RTOL_L2
    # point depos land whole in one bin
    assert g[int(7.0 / 1.25), int(10.0 / 0.5)] == pytest.approx(100.0, rel=1e-6)
    empty = inputs.Depos(*(np.zeros(0, np.float32) for _ in range(5)))
    assert not gpu_raster(P, empty).any()


def test_nonfinite_depos_counter():
    """lar_depos_nonfinite counts the depos the raster skips: any NaN or
    infinite field, in any of the five arrays; 0 for an empty set."""
    torch, lar = _torch(), _lar()
    rng = np.random.default_rng(23)
    n = 300_001
    arrs = [rng.standard_normal(n).astype(np.float32) for _ in range(5)]
    for k, a in enumerate(arrs):
        idx = rng.choice(n, 700 + 100 * k, replace=False)
        a[idx] = rng.choice(np.array([np.nan, np.inf, -np.inf], np.float32), idx.size)
    dep = inputs.Depos(*arrs)
    expect = int(np.sum(~np.all(np.isfinite(np.stack(arrs)), axis=0)))
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    assert lar.depos_nonfinite(lar.DeviceDepos.from_host(dep), out).item() == expect
    # the count is written, not accumulated
    assert lar.depos_nonfinite(lar.DeviceDepos.from_host(dep), out).item() == expect
    empty = inputs.Depos(*(np.zeros(0, np.float32) for _ in range(5)))
    assert lar.depos_nonfinite(lar.DeviceDepos.from_host(empty), out).item() == 0


def test_atomic_probe_counts():
    """The float-atomic rate probe adds exactly 1 to every float of each
    hashed 64-float segment, per call, and leaves the tail past the last
    whole segment alone."""
    torch, lar = _torch(), _lar()
    n, n_seg = 64 * 1000 + 17, 50_000
    buf = torch.zeros(n, device="cuda")
    lar.atomic_probe(buf, n_seg)
    lar.atomic_probe(buf, n_seg)
    sg = np.arange(n_seg, dtype=np.uint64)
    with np.errstate(over="ignore"):
        slot = ((sg * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(17)) % np.uint64(1000)
    expect = np.zeros(n, np.float32)
    expect[:64000] = np.repeat(2.0 * np.bincount(slot.astype(np.int64), minlength=1000), 64)
    assert np.array_equal(buf.cpu().numpy(), expect)
    lar.atomic_probe(buf, 0)
    torch.cuda.synchronize()


def test_philox_probe_sums():
    """The Philox rate probe's per-thread sums equal the oracle's Philox4x32-10
    uniforms of the same counters, added in the same order (bit-exact)."""
    torch, lar = _torch(), _lar()
    n_threads, n_blocks = 512, 3001
    out = torch.full((n_threads,), -1.0, dtype=torch.float64, device="cuda")
    lar.philox_probe(out, n_blocks)
    torch.cuda.synchronize()
    ref = np.zeros(n_threads)
    key = [0x12345678, 0x9ABCDEF0]
    for i in range(n_blocks):
        o = oracle.philox([i & 0xFFFFFFFF, 0x5EED, i >> 32, 0], key)
        ref[i % n_threads] += oracle.u53(o[0], o[1])
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("rows,n_in,n_out,per_cu", [(1, 6000, 3073, 1), (37, 6000, 3073, 2), (600, 1024, 513, 3),
                                                    (5, 6144, 3073, 4)])
def test_row_copy_probe_rows(rows, n_in, n_out, per_cu):
    """The row-copy probe writes pair k of each input row to element k of
    its output row (the last pair repeated past n_in/2) and nothing past
    n_out."""
    torch, lar = _torch(), _lar()
    src = torch.randn(rows, n_in, device="cuda")
    dst = torch.full((rows, 2 * n_out + 6), -7.0, device="cuda")
    lar.row_copy_probe(src, dst, n_out, per_cu)
    torch.cuda.synchronize()
    got, ref = dst.cpu().numpy(), src.cpu().numpy()
    half = min(n_in // 2, n_out)
    assert np.array_equal(got[:, :2 * half], ref[:, :2 * half])
    if n_out > n_in // 2:
        tail = got[:, 2 * half:2 * n_out].reshape(rows, -1, 2)
        assert np.array_equal(tail, np.broadcast_to(ref[:, None, n_in - 2:n_in], tail.shape))
    assert (got[:, 2 * n_out:] == -7.0).all()


def test_raster_accumulates():
    torch, lar = _torch(), _lar()
    ev = inputs.cfg0_event()
    P, dep = ev.planes[0], ev.depos[0]
    D = lar.DeviceDepos.from_host(dep)
    grid = torch.ones((P.n_rows, P.n_ticks), dtype=torch.float32, device="cuda")
    lar.raster(P, D, 3.0, None, grid)
    lar.raster(P, D, 3.0, None, grid)
    ref = 1.0 + 2.0 * oracle.raster_mean(P, dep)
    assert rel_l2(grid.cpu().numpy(), ref) < RTOL_L2


# ------------------------------------------------------------------ convolution

FFT_CASES = [
    dict(n_wires=5, n_ticks=40, n_imp=2, nt_fft=48, nw_fft=9),
    dict(n_wires=7, n_ticks=100, n_imp=3, nt_fft=108, nw_fft=12),
    dict(n_wires=4, n_ticks=18, n_imp=1, nt_fft=18, nw_fft=4),           # wrap in both axes
    dict(n_wires=64, n_ticks=1024, n_imp=10, nt_fft=1024, nw_fft=96),    # tiny plane shape
    dict(n_wires=30, n_ticks=1000, n_imp=10, nt_fft=1024, nw_fft=864),
    dict(n_wires=21, n_ticks=6000, n_imp=10, nt_fft=6144, nw_fft=512),
    dict(n_wires=3, n_ticks=2, n_imp=1, nt_fft=2, nw_fft=3),
    dict(n_wires=10, n_ticks=16000, n_imp=2, nt_fft=16384, nw_fft=16),
    dict(n_wires=1000, n_ticks=64, n_imp=2, nt_fft=64, nw_fft=1024),    # the largest wire FFT accepted
    dict(n_wires=8, n_ticks=96, n_imp=40, nt_fft=96, nw_fft=12),        # many impact offsets per wire
]


@pytest.mark.parametrize("case", FFT_CASES)
def test_fftconv_random_grid_and_spectrum(case):
    P = inputs.Plane(**case)
    g = inputs.random_grid(P, 11, density=0.3)
    R = inputs.random_spectrum(P, 12)
    w = gpu_fftconv(P, g, R)
    ref = oracle.conv_fft(P, g, R)
    assert np.isfinite(w).all()
    assert rel_l2(w, ref) < RTOL_L2
    assert np.max(np.abs(w - ref)) <= RTOL_L2 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", [dict(n_wires=21, n_ticks=6144, n_imp=4, nt_fft=6144, nw_fft=512),
                                  dict(n_wires=30, n_ticks=1024, n_imp=3, nt_fft=1024, nw_fft=864)])
@pytest.mark.parametrize("column", ["dc", "nyquist"])
def test_fftconv_dc_and_nyquist_columns(case, column):
    """Grids whose every row is constant (all of its spectrum in the DC
    column) or alternates in sign tick by tick (all in the Nyquist column,
    n_ticks = Tf): an error in the wire pass's first or last column tile
    (the Nyquist column is a tile of its own at Wf 512 with 16-column tiles)
    then dominates the waveforms instead of hiding among 3073 columns."""
    P = inputs.Plane(**case)
    rng = np.random.default_rng(17)
    amp = rng.standard_normal((P.n_rows, 1)).astype(np.float32)
    sign = np.ones(P.n_ticks, np.float32) if column == "dc" else (-1.0) ** np.arange(P.n_ticks, dtype=np.float32)
    g = (amp * sign[None, :]).astype(np.float32)
    R = inputs.random_spectrum(P, 18)
    w = gpu_fftconv(P, g, R)
    ref = oracle.conv_fft(P, g, R)
    assert rel_l2(w, ref) < RTOL_L2
    assert np.max(np.abs(w - ref)) <= RTOL_L2 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", [dict(n_wires=64, n_ticks=1024, nt_fft=1024, nw_fft=96, kind="unipolar"),
                                  dict(n_wires=480, n_ticks=6000, nt_fft=6144, nw_fft=512, kind="unipolar"),
                                  dict(n_wires=800, n_ticks=6000, nt_fft=6144, nw_fft=864, kind="bipolar"),
                                  dict(n_wires=6, n_ticks=50, n_imp=3, nt_fft=54, nw_fft=8, half_w=10)])
def test_response_spectrum(case):
    kind = case.pop("kind", "unipolar")
    P = inputs.Plane(**case)
    r = inputs.response_time(P.n_imp, P.half_w, min(200, P.n_ticks), kind)
    resp = _lar().spectrum_from_time(P, r).cpu().numpy()
    ref = oracle.response_spectrum(P, r)
    got = resp[..., 0] + 1j * resp[..., 1]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < RTOL_L2
    assert np.max(np.abs(got - ref)) <= RTOL_L2 * np.max(np.abs(ref))


def test_fftconv_equals_direct_sum_tiny():
    """GPU convolution against the brute-force Eq. (1) sum."""
    P = inputs.Plane(n_wires=9, n_ticks=60, n_imp=3, nt_fft=64, nw_fft=16, half_w=3)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((3, 7, 12)).astype(np.float32)
    S = rng.standard_normal((P.n_rows, P.n_ticks)).astype(np.float32)
    resp = _lar().spectrum_from_time(P, r).cpu().numpy()
    w = gpu_fftconv(P, S, resp)
    ref = oracle.conv_direct(P, r, S)
    assert rel_l2(w, ref) < RTOL_L2
    assert np.max(np.abs(w - ref)) <= RTOL_L2 * np.max(np.abs(ref))


# ------------------------------------------------------------------ end to end

def _sim_plane(P, dep, resp, fluct=None):
    torch, lar = _torch(), _lar()
    D = lar.DeviceDepos.from_host(dep)
    wave = torch.empty((P.n_wires, P.n_ticks), dtype=torch.float32, device="cuda")
    ws = lar.workspace(lar.sim_plane_workspace(P, len(dep), fluct))
    lar.sim_plane(P, D, 3.0, fluct, resp, wave, ws)
    torch.cuda.synchronize()
    return wave.cpu().numpy()


@pytest.mark.parametrize("cfg", ["cfg0", "cfg1"])
def test_sim_plane_mean(cfg):
    ev = inputs.cfg0_event() if cfg == "cfg0" else inputs.cfg1_event()
    P, dep = ev.planes[0], ev.depos[0]
    r = inputs.response_time(P.n_imp, P.half_w, 200, P.kind)
    resp_dev = _lar().spectrum_from_time(P, r)
    w = _sim_plane(P, dep, resp_dev)
    ref = oracle.sim_plane_mean(P, dep, oracle.response_spectrum(P, r))
    assert rel_l2(w, ref) < RTOL_L2
    assert np.max(np.abs(w - ref)) <= RTOL_L2 * np.max(np.abs(ref))


# ------------------------------------------------------------------ fluctuation

def _injected(n, seed=5):
    rng = np.random.default_rng(seed)
    regime = rng.integers(0, 6, n)
    q = np.where(regime < 2, rng.uniform(1, 60, n), np.where(regime < 4, rng.uniform(100, 5e3, n),
                                                            10 ** rng.uniform(3, 6, n)))
    q = (q * np.where(rng.uniform(size=n) < 0.1, -1, 1)).astype(np.float32)
    p = np.where(regime % 2 == 0, 10 ** rng.uniform(-6, -1, n), rng.uniform(0, 1, n))
    p[:5] = [0.0, 1.0, 0.5, 1e-300, 1 - 1e-12]
    ctr = rng.integers(0, 2 ** 32, (n, 3), dtype=np.uint64).astype(np.uint32)
    return q, p, ctr


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_sampler_bit_exact(mode):
    torch, lar = _torch(), _lar()
    q, p, ctr = _injected(200_000, seed=mode)
    out = torch.empty(len(q), dtype=torch.float32, device="cuda")
    lar.sample_counts(mode, torch.from_numpy(q).cuda(), torch.from_numpy(p).cuda(),
                      torch.from_numpy(ctr).cuda().contiguous(), 3, 0xDEADBEEF12345, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.sample_counts(mode, q, p, ctr, 3, 0xDEADBEEF12345)
    mism = np.flatnonzero(got != ref)
    assert len(mism) == 0, (len(mism), q[mism[:5]], p[mism[:5]], got[mism[:5]], ref[mism[:5]])


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_raster_fluct_cfg0_matches_oracle_keys(mode):
    """Same keys, p equal up to FP32 rounding: nearly every bin is identical,
    and the totals agree with the mean path within the statistical spread
    (binomial, Poisson; the rounded, clipped normal approximation is biased
    at small means, so its total is compared with the oracle's)."""
    ev = inputs.cfg0_event()
    P, dep = ev.planes[0], ev.depos[0]
    seed = inputs.SEED0
    g = gpu_raster(P, dep, fluct=(mode, seed, 0, 2))
    ref = oracle.raster_fluct(P, dep, mode=mode, seed=seed, event=0, plane_id=2)
    assert np.array_equal(g, np.round(g))
    same = np.mean(g == ref)
    assert same > 0.9999, same
    if mode == 3:
        assert abs(g.sum() - ref.sum()) < 1e-4 * abs(ref.sum())
        return
    mean = oracle.raster_mean(P, dep)
    # independent bins: Var(sum) = sum N p (1 - p) <= sum N p (binomial), = sum |q| p (Poisson)
    z = (g.sum() - mean.sum()) / math.sqrt(mean.sum())
    assert abs(z) < 5


def test_fluct_chi2_mean_and_variance():
    """Fluctuated grids over many seeds: per-bin mean = mean grid, variance =
    N p (1 - p) (binomial), as chi-square over the bins."""
    torch, lar = _torch(), _lar()
    P = inputs.Plane(n_wires=6, n_ticks=64, n_imp=10)
    dep = inputs.random_depos(P, 20, seed=4)
    dep.q[:] = 300.0
    D = lar.DeviceDepos.from_host(dep)
    reps = 400
    grids = torch.zeros((reps, P.n_rows, P.n_ticks), dtype=torch.float32, device="cuda")
    ws = lar.workspace(lar.raster_workspace(P, len(dep), (1, 0, 0, 0)))
    for s in range(reps):
        lar.raster(P, D, 3.0, (1, 1000 + s, 0, 0), grids[s], ws)
    G = grids.double().cpu().numpy()
    # per-depo bins are independent: Var of the sum = sum over depos of N p (1-p)
    var = np.zeros((P.n_rows, P.n_ticks))
    mean = np.zeros_like(var)
    for i in range(len(dep)):
        mi = oracle.raster_mean(P, dep.take(slice(i, i + 1)))
        mean += mi
        var += mi * (1 - mi / 300.0)
    sel = mean > 5
    zm = (G.mean(0)[sel] - mean[sel]) / np.sqrt(var[sel] / reps)
    chi2 = float((zm ** 2).sum())
    from scipy import stats
    assert stats.chi2.sf(chi2, sel.sum()) > 1e-4
    ratio = G.var(0, ddof=1)[sel] / var[sel]
    assert abs(np.mean(ratio) - 1) < 0.05


@pytest.mark.parametrize("mode", [1, 2])
def test_fluct_queue_capacity_does_not_change_counts(mode):
    """Bins beyond the rejection samplers' fast region go through the
    workspace queue; with a queue of zero or a few entries they are redrawn
    by the flagged-sub-chunk kernel instead.  Counts are integers: bit-identical."""
    ev = inputs.cfg0_event()
    P, dep = ev.planes[0], ev.depos[0]
    fl = (mode, 99, 4, 1)
    lar = _lar()
    full = gpu_raster(P, dep, fluct=fl)
    n = len(dep)
    fixed = 256 + ((n + 15) // 16 + 255) // 256 * 256
    for nb in (fixed, fixed + 16 * 37):
        assert np.array_equal(gpu_raster(P, dep, fluct=fl, ws_bytes=nb), full)
    with pytest.raises(lar.LarError):
        gpu_raster(P, dep, fluct=fl, ws_bytes=fixed - 256)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_fluct_wide_depos_with_queue_overflow(mode):
    """Depos wider than the hot raster kernel's weight slots (16 ticks, 32
    impact rows), mixed with regular ones in the same sub-chunks: the oracle's
    counts on nearly every bin, and the same counts with a queue of a few
    entries or none (the flagged sub-chunks are then drawn by one kernel for
    both reasons)."""
    P = inputs.Plane(n_wires=24, n_ticks=400, n_imp=10)
    dep = inputs.random_depos(P, 240, seed=12)
    dep.sigma_t[::3] *= 4.0
    dep.sigma_x[1::3] *= 3.0
    fl = (mode, 77, 0, 1)
    full = gpu_raster(P, dep, fluct=fl)
    ref = oracle.raster_fluct(P, dep, mode=mode, seed=77, event=0, plane_id=1)
    assert np.array_equal(full, np.round(full))
    nz = (full != 0) | (ref != 0)
    assert np.mean(full[nz] == ref[nz]) > 0.999
    n = len(dep)
    fixed = 256 + ((n + 15) // 16 + 255) // 256 * 256
    for nb in (fixed, fixed + 16 * 37):
        assert np.array_equal(gpu_raster(P, dep, fluct=fl, ws_bytes=nb), full)


def test_fluct_point_charges_large_q():
    """Point-like and high-charge depos: every bin in the rejection regime."""
    P = inputs.Plane(n_wires=16, n_ticks=200, n_imp=10)
    dep = inputs.random_depos(P, 300, seed=8, sigma_scale=0.5)
    dep.q[:] = (10 ** np.random.default_rng(2).uniform(4, 6, len(dep))).astype(np.float32)
    g = gpu_raster(P, dep, fluct=(1, 5, 0, 0))
    ref = oracle.raster_fluct(P, dep, mode=1, seed=5, event=0, plane_id=0)
    assert np.mean(g == ref) > 0.999
    assert g.sum() == pytest.approx(ref.sum(), rel=1e-3)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_raster_fluct_cfg1_full_size(mode):
    """The headline event (500k depos, 480 x 10 rows x 6000 ticks) in the
    launch configuration the benchmark times: integer counts summed in
    float32 are exact, so every bin whose p rounds the same on both sides is
    identical to the oracle's."""
    ev = inputs.cfg1_event()
    P, dep = ev.planes[0], ev.depos[0]
    seed = inputs.SEED0 + 100
    lar = _lar()
    fl = (mode, seed, 0, 2)
    g = gpu_raster(P, dep, fluct=fl, ws_bytes=lar.sim_plane_workspace(P, len(dep), fl)
                   - lar.sim_plane_workspace(P))
    ref = oracle.raster_fluct(P, dep, mode=mode, seed=seed, event=0, plane_id=2)
    assert np.array_equal(g, np.round(g))
    nz = (g != 0) | (ref != 0)
    same = np.mean(g[nz] == ref[nz])
    assert same > 0.9999, same
    assert abs(g.sum() - ref.sum()) < 1e-4 * abs(ref.sum())
