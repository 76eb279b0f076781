"""Benchmark: depositions/s of the LArTPC signal-simulation hot path on one
MI355X (raster + scatter-add + FFT convolution, forward and forward+backward).

Headline (`value`; one step = one plane-frame): the full collection plane,
480 wires x 6000 ticks (time FFT 6144, wire FFT 512), 10 impact positions
per pitch, 500k depositions from 60 seeded cosmic-muon-like segments
crossing a 3.6 m drift, binomial fluctuation, FP32 (FP64 sampler).  Inputs
and the response spectrum are resident on the device before timing.

Every leg times each repetition with HIP events on the stream the library
launches on and reports the median of the repetitions after warm-ups.
Extra objects of the same JSON line:
  modes        the headline plane with the mean patch, Poisson and the
               normal approximation instead of the binomial;
  three_plane  one event of the three-plane readout (U, V: 800 wires,
               bipolar, Wf 864; W: 480 wires; 2M depos incl. 100k points),
               three lar_sim_plane calls, and as a 3-item batch plan; the
               U plane's per-stage times and FFT roofline;
  batched      64 events x 3 planes with log-uniform depo counts: the batch
               plan (waves bounded by a workspace budget, hipGraph) against
               192 sequential lar_sim_plane calls and against the streams
               executor on 1, 2, 4 and 8 streams;
  fwd_bwd      16 events x 200k depos on the collection plane, mean path,
               forward + MSE + backward: 16 sequential autograd steps, and
               the batched forward + batched backward plan;
  cpu_baseline the FP64 oracle on the host's cores (and on one thread).

Profiling aids (each prints its own JSON and exits): --calib (a 1 GiB copy
for scaling the PMC byte counters), --atomic-peak (the peak rate of the
raster's scattered float atomics), --philox-peak (the rate of its per-bin
Philox draw), --copy-floor (the memory floor of the
time R2C's access pattern), --leg NAME (one extra leg alone).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# full-rate 32-bit VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# algorithmic integer work of one drawn bin: one Philox4x32-10 block
# (10 rounds x (2 wide multiplies = 4 word products + 4 XORs) + 9 key
# bumps x 2 adds = 98) and the 52-bit uniform (2 shifts, 2 conversions,
# 1 multiply, 2 adds, 1 scale = 8)
OPS_PER_BIN = 98 + 8
STAGES = ["fill", "raster", "raster_tail", "r2c", "wire", "c2r"]
BATCH_BUDGET = 24 << 30      # workspace budget of the batch plan (bytes)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def med(xs):
    return statistics.median(xs)


def spec_ld(P):
    return (P.nt_fft // 2 + 1 + 15) // 16 * 16


def algorithmic_bytes(P, n_resp_reads=1.0, items=1):
    """HBM bytes each FFT-path kernel must move for `items` plane-frames of
    plane P (read inputs once, write outputs once; the response spectrum
    read n_resp_reads times in all)."""
    R, N, F = P.n_rows, P.n_ticks, P.nt_fft // 2 + 1
    return {
        "fill": items * R * N * 4,
        "r2c": items * (R * N * 4 + R * F * 8),
        "wire": items * (R * F * 8 + P.n_wires * F * 8) + n_resp_reads * P.n_imp * P.nw_fft * F * 8,
        "c2r": items * (P.n_wires * F * 8 + P.n_wires * N * 4),
    }


def count_bins(P, dep, nsigma):
    """Bins of every depo's window (the raster's units of work), counted on the host."""
    import numpy as np

    def axis(mu, sg, org, wd, nb):
        mu = mu.astype(np.float64)
        sg = sg.astype(np.float64)
        ns = float(np.float32(nsigma))
        point = sg < 1e-6 * wd
        f = np.floor((mu - org) / wd)
        n_pt = ((f >= 0) & (f < nb)).astype(np.int64)
        lo = np.maximum(np.floor((mu - ns * sg - org) / wd), 0)
        hi = np.minimum(np.floor((mu + ns * sg - org) / wd), nb - 1)
        n = np.where(lo <= hi, hi - lo + 1, 0).astype(np.int64)
        return np.where(point, n_pt, n)

    q, t, x, st, sx = dep.arrays()
    ok = np.isfinite(q) & np.isfinite(t) & np.isfinite(x) & np.isfinite(st) & np.isfinite(sx)
    nt = axis(t, st, float(np.float32(P.t0)), float(np.float32(P.tick)), P.n_ticks)
    xl = float(np.float32(P.x0)) - float(np.float32(P.pitch)) / 2.0
    nx = axis(x, sx, xl, float(np.float32(P.pitch)) / P.n_imp, P.n_rows)
    return int(np.sum(np.where(ok, nt * nx, 0)))


def load_traffic(path):
    """Measured HBM bytes per launch of each stage's kernel (rocprofv3
    FETCH_SIZE / WRITE_SIZE, scaled by a plain copy's reading), kept only for
    stages whose kernel sources are unchanged since the counters were taken."""
    from paper_2203_02479_amd import profsum
    try:
        data = json.load(open(path))
    except Exception:
        return {}
    out = {}
    for stage, rec in data.items():
        if stage.startswith("_") or not isinstance(rec, dict):
            continue
        if rec.get("source") == profsum.source_digest(stage):
            out[stage] = rec["bytes"]
    return out


def copy_calibration(torch):
    """A plain copy kernel of known size (an elementwise multiply by one: reads
    1 GiB, writes 1 GiB), for scaling the PMC byte counters."""
    n = 1 << 28                                   # 1 GiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    log(f"calibration: copied {n * 4} bytes 5 times")


def atomic_peak(torch, lar, reps=20):
    """Peak rate of scattered 64-float wave atomics (the raster's tile-flush
    access) over a buffer the size of the collection plane's impact-resolved
    raster target (4800 rows x 6000 ticks)."""
    n = 4800 * 6000
    buf = torch.zeros(n, device="cuda")
    n_seg = 1 << 22
    ms = time_reps(torch, lambda: lar.atomic_probe(buf, n_seg), 3, reps)
    med_ms = float(statistics.median(ms))
    out = {"segments": n_seg, "floats": n_seg * 64, "buffer_bytes": n * 4, "reps": reps,
           "median_ms": round(med_ms, 4), "wave_atomics_per_s": n_seg / med_ms * 1e3,
           "float_atomics_per_s": n_seg * 64 / med_ms * 1e3}
    torch.cuda.synchronize()
    total = float(buf.double().sum().item())
    expect = float(n_seg) * 64 * (reps + 3)
    if total != expect:
        raise RuntimeError(f"atomic probe: buffer sum {total} != {expect}")
    return out


def philox_peak(torch, lar, reps=20):
    """Rate of the raster's per-bin draw (one Philox4x32-10 block and its
    52-bit uniform) with every CU full: 2048 threads per CU, 2^28 blocks."""
    n_threads, n_blocks = 256 * 2048, 1 << 28
    out = torch.empty(n_threads, dtype=torch.float64, device="cuda")
    ms = med(time_reps(torch, lambda: lar.philox_probe(out, n_blocks), 3, reps))
    mean = float(out.sum().item()) / n_blocks
    if abs(mean - 0.5) > 1e-3:
        raise RuntimeError(f"philox probe: mean uniform {mean}")
    rate = n_blocks / (ms * 1e-3)
    return {"blocks": n_blocks, "threads": n_threads, "reps": reps, "median_ms": round(ms, 4),
            "blocks_per_s": rate, "ops_per_s": rate * OPS_PER_BIN,
            "frac_of_valu_peak": round(rate * OPS_PER_BIN / (VALU_PEAK_GOPS * 1e9), 4),
            "mean_uniform": mean}


def copy_floor(torch, lar, reps=30):
    """Memory floors of the time R2C's bytes at the collection plane's 4800
    rows and the induction plane's 8000 rows (6000 ticks, Tf 6144): the
    library's row-copy probe (the transform's grid and access pattern, no
    transform) at 1-4 workgroups per CU, and a flat device copy of the same
    byte count."""
    out = {}
    n_in, n_out, ld_out = 6000, 3073, 3088
    for rows in (4800, 8000):
        src = torch.randn(rows, n_in, device="cuda")
        dst = torch.zeros(rows, 2 * ld_out, device="cuda")
        nbytes = rows * (n_in * 4 + n_out * 8)
        rec = {"bytes": nbytes}
        for per in (1, 2, 3, 4):
            ms = med(time_reps(torch, lambda: lar.row_copy_probe(src, dst, n_out, per), 3, reps))
            rec[f"row_copy_{per}_per_cu_us"] = round(ms * 1e3, 2)
            rec[f"row_copy_{per}_per_cu_gbs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
        if not torch.equal(dst[:, :n_in], src):
            raise RuntimeError("row copy probe: output rows differ from the input rows")
        half = nbytes // 2 // 4
        a = torch.randn(half, device="cuda")
        b = torch.empty_like(a)
        ms = med(time_reps(torch, lambda: b.copy_(a), 3, reps))
        rec["flat_copy_us"] = round(ms * 1e3, 2)
        rec["flat_copy_gbs"] = round(2 * half * 4 / (ms * 1e-3) / 1e9, 1)
        out[f"{rows}_rows"] = rec
        del src, dst, a, b
        torch.cuda.empty_cache()
    return out


def time_reps(torch, fn, warmup, reps, stream=None):
    """Per-repetition times (ms) of fn() with HIP events on `stream`."""
    stream = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


TUNED = {}


def tune_plane(args, P):
    """Time the candidate FFT schedules of this plane shape and register the
    fastest (outside every timed region)."""
    from paper_2203_02479_amd import autotune
    key = autotune.shape_key(P)
    if key in TUNED or args.no_tune:
        return
    out = autotune.tune(P, reps=5, cache=False)
    TUNED[key] = {**out["schedule"], "ms": round(out["rows_ms"] + out["wire_ms"], 4),
                  "builtin_ms": round(out["default_ms"], 4), "candidates": out["candidates"]}
    log(f"bench: schedule {key} {json.dumps(TUNED[key])}")


def tune_raster(args, P, D, fl):
    """Time the raster tiles of this plane shape on these depositions and
    register the fastest (outside every timed region)."""
    from paper_2203_02479_amd import autotune
    key = autotune.shape_key(P)
    if args.no_tune or TUNED.get(key, {}).get("raster_ms"):
        return
    out = autotune.tune_raster(P, D, inputs_mod().NSIGMA, fl, reps=5, cache=False)
    entry = TUNED.setdefault(key, {})
    entry["raster_tile"] = out["raster_tile"]
    entry["raster_ms"] = {str(k): round(v, 4) for k, v in out["ms"].items()}
    log(f"bench: raster tile {key} {json.dumps(entry['raster_ms'])} -> {out['raster_tile']}")


def inputs_mod():
    from paper_2203_02479_amd import inputs
    return inputs


def fft_roofline(nbytes, per):
    out = {}
    for k in ("r2c", "wire", "c2r", "fill"):
        if k in per and per[k] > 0:
            ach = nbytes[k] / (per[k] * 1e-3) / 1e9
            out[k] = {"achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                      "algorithmic_bytes": int(nbytes[k]), "avg_ms": round(per[k], 5)}
    return out


# ------------------------------------------------------------------ headline

def leg_forward(args, torch, lar, inputs, np, mode, K, warmup, with_stages=True):
    ev = inputs.cfg1_event()
    P, dep = ev.planes[0], ev.depos[0]
    r = inputs.response_time(P.n_imp, P.half_w, inputs.RESP_TICKS, P.kind)
    D = lar.DeviceDepos.from_host(dep)
    resp = lar.spectrum_from_time(P, r)
    tune_plane(args, P)
    seed = inputs.SEED0 + 100
    fl0 = (mode, seed, 0, 2) if mode else None
    tune_raster(args, P, D, (1, seed, 0, 2))   # the tile of the headline (binomial) workload
    ws = lar.workspace(lar.sim_plane_workspace(P, len(dep), fl0))
    wave = torch.empty((P.n_wires, P.n_ticks), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    counter = [0]

    def step():
        i = counter[0]
        counter[0] += 1
        fl = (mode, seed, i, 2) if mode else None
        lar.sim_plane(P, D, inputs.NSIGMA, fl, resp, wave, ws, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev_start = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    stage = [[torch.cuda.Event(enable_timing=True) for _ in STAGES] for _ in range(K)]
    for row in stage:                              # materialise the HIP events
        for e in row:
            e.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        ev_start[i].record(stream)
        if with_stages:
            lar.set_stage_events(stage[i])
        step()
        if not with_stages:
            stage[i][-1].record(stream)
    lar.set_stage_events(None)
    torch.cuda.synchronize()
    host_s = time.perf_counter() - t0
    steps_ms = [ev_start[i].elapsed_time(stage[i][-1]) for i in range(K)]
    per = {}
    if with_stages:
        for s_, n in enumerate(STAGES):
            per[n] = med([(ev_start[i] if s_ == 0 else stage[i][s_ - 1]).elapsed_time(stage[i][s_])
                          for i in range(K)])
    return P, dep, r, seed, steps_ms, per, host_s


# ------------------------------------------------------------------ three planes

def leg_three_plane(args, torch, lar, inputs, np):
    log("bench: three-plane event (2M depos)")
    ev = inputs.cfg2_event()
    seed = inputs.SEED0 + 200
    planes = ev.planes
    rt = [inputs.response_time(p.n_imp, p.half_w, inputs.RESP_TICKS, p.kind) for p in planes]
    resps = [lar.spectrum_from_time(p, r) for p, r in zip(planes, rt)]
    for p in (planes[0], planes[2]):
        tune_plane(args, p)
    Ds = [lar.DeviceDepos.from_host(d) for d in ev.depos]
    fl = (1, seed, 0, 0)
    tune_raster(args, planes[0], Ds[0], fl)
    wss = [lar.workspace(lar.sim_plane_workspace(p, len(d), fl)) for p, d in zip(planes, ev.depos)]
    waves = [torch.empty((p.n_wires, p.n_ticks), device="cuda") for p in planes]
    n_depo = len(ev.depos[0])

    def three():
        for pl in range(3):
            lar.sim_plane(planes[pl], Ds[pl], inputs.NSIGMA, (1, seed, 0, pl), resps[pl], waves[pl], wss[pl])

    reps = max(10, args.steps // 2)
    ms = med(time_reps(torch, three, 3, reps))
    # per-stage times of the U plane (800 wires, Wf 864): the FFT stages at
    # this shape against their algorithmic bytes
    stream = torch.cuda.current_stream()
    stage = [[torch.cuda.Event(enable_timing=True) for _ in STAGES] for _ in range(reps)]
    start = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for row in stage:
        for e in row:
            e.record(stream)
    for _ in range(3):
        three()
    torch.cuda.synchronize()
    for i in range(reps):
        start[i].record(stream)
        lar.set_stage_events(stage[i])
        lar.sim_plane(planes[0], Ds[0], inputs.NSIGMA, (1, seed, 0, 0), resps[0], waves[0], wss[0], stream)
    lar.set_stage_events(None)
    torch.cuda.synchronize()
    per_u = {n: med([(start[i] if s_ == 0 else stage[i][s_ - 1]).elapsed_time(stage[i][s_]) for i in range(reps)])
             for s_, n in enumerate(STAGES)}
    roof_u = fft_roofline(algorithmic_bytes(planes[0]), per_u)
    # the same event as a 3-item batch plan (U, V share a type)
    del wss
    types = [planes[0], planes[2]]
    items, cat, off, woff = [], [], 0, 0
    for pl in range(3):
        pt = 0 if pl < 2 else 1
        items.append((pt, 0, pl, off, len(ev.depos[pl]), woff))
        cat.append(ev.depos[pl])
        off += len(ev.depos[pl])
        woff += types[pt].n_wires * types[pt].n_ticks
    catd = lar.DeviceDepos(*(torch.as_tensor(np.concatenate([c.arrays()[k] for c in cat])).cuda()
                             for k in range(5)))
    wave = torch.empty(woff, device="cuda")
    ws = lar.workspace(lar.batch_workspace(types, items, fl))
    plan = lar.Batch(types, [resps[0], resps[2]], catd, inputs.NSIGMA, fl, items, wave, ws, use_graph=True)
    ms_b = med(time_reps(torch, plan.run, 3, reps))
    plan.close()
    bins = sum(count_bins(p, d, inputs.NSIGMA) for p, d in zip(planes, ev.depos))
    nb = [algorithmic_bytes(p) for p in planes]
    fft_bytes = sum(sum(v for k, v in b.items() if k != "fill") for b in nb)
    return {"workload": "one event of the three-plane readout: U, V 800 wires (bipolar, Wf 864), W 480 wires "
                        "(unipolar), 6000 ticks, 1.9M track + 100k point depos (q 1e2-1e5), binomial fluctuation",
            "depos": n_depo, "bins": bins, "reps": reps,
            "ms_per_event": round(ms, 4), "depos_per_s": round(n_depo / (ms * 1e-3), 1),
            "plane_frames_per_s": round(3e3 / ms, 2),
            "batch_plan_ms_per_event": round(ms_b, 4),
            "batch_plan_depos_per_s": round(n_depo / (ms_b * 1e-3), 1),
            "fft_algorithmic_bytes": int(fft_bytes),
            "u_plane_kernel_ms": {k: round(v, 5) for k, v in per_u.items()},
            "roofline_fft_u_plane": roof_u}


# ------------------------------------------------------------------ batch

def leg_batched(args, torch, lar, inputs, np):
    log("bench: batched, 64 events x 3 planes")
    evs = inputs.cfg3_events()
    planes = [evs[0].planes[0], evs[0].planes[2]]              # U/V geometry (type 0), W (type 1)
    rt = [inputs.response_time(p.n_imp, p.half_w, inputs.RESP_TICKS, p.kind) for p in planes]
    resps = [lar.spectrum_from_time(p, r) for p, r in zip(planes, rt)]
    for p in planes:
        tune_plane(args, p)
    items, chunks, off, woff = [], [], 0, 0
    for e, ev in enumerate(evs):
        for pl in range(3):
            pt = 0 if pl < 2 else 1
            d = ev.depos[pl]
            items.append((pt, e, pl, off, len(d), woff))
            chunks.append(d)
            off += len(d)
            woff += planes[pt].n_wires * planes[pt].n_ticks
    cat = [np.concatenate([c.arrays()[k] for c in chunks]) for k in range(5)]
    D = lar.DeviceDepos(*(torch.as_tensor(a).cuda() for a in cat))
    seed = inputs.SEED0 + 300
    fl = (1, seed, 0, 0)
    wave = torch.empty(woff, device="cuda")
    full = lar.batch_workspace(planes, items, fl)
    nbytes = min(full, BATCH_BUDGET)
    log(f"bench: batch workspace {nbytes / 2**30:.1f} GiB (all items at once: {full / 2**30:.1f} GiB)")
    ws = lar.workspace(nbytes)
    plan = lar.Batch(planes, resps, D, inputs.NSIGMA, fl, items, wave, ws, use_graph=True)
    n_waves, wave_items = plan.waves()
    reps = max(10, args.steps // 2)
    ms_batch = med(time_reps(torch, plan.run, 3, reps))
    plan.close()
    del ws
    torch.cuda.empty_cache()
    # sequential single-plane calls on the same device buffers
    nmax = max(it[4] for it in items)
    ws1 = lar.workspace(max(lar.sim_plane_workspace(p, nmax, fl) for p in planes))
    views = []
    for (pt, e, pl, o, n, wo) in items:
        dd = lar.DeviceDepos(*(getattr(D, f)[o:o + n] for f in ("q", "t", "x", "sigma_t", "sigma_x")))
        views.append((planes[pt], dd, resps[pt], wave[wo:wo + planes[pt].n_wires * planes[pt].n_ticks], e, pl))

    def seq():
        for P, dd, rr, w, e, pl in views:
            lar.sim_plane(P, dd, inputs.NSIGMA, (1, seed, e, pl), rr, w, ws1)

    ms_seq = med(time_reps(torch, seq, 1, max(5, reps // 2)))
    del ws1
    torch.cuda.empty_cache()
    # the streams executor
    streams_ms = {}
    for ns in (1, 2, 4, 8):
        sts = [torch.cuda.Stream() for _ in range(ns)]
        wss = lar.workspace(lar.sim_streams_workspace(planes, items, fl, ns))
        fn = lambda: lar.sim_streams(planes, resps, D, inputs.NSIGMA, fl, items, wave, sts, wss)
        streams_ms[ns] = round(med(time_reps(torch, fn, 1, max(5, reps // 2))), 3)
        del wss
        torch.cuda.empty_cache()
    n_depo = sum(len(ev.depos[0]) for ev in evs)
    bins = sum(count_bins(planes[it[0]], c, inputs.NSIGMA) for it, c in zip(items, chunks))
    # algorithmic FFT bytes of the batch: every item's rows once, each type's
    # response once per wave of that type
    waves_of = {0: 0, 1: 0}
    counts = {0: sum(1 for it in items if it[0] == 0), 1: sum(1 for it in items if it[0] == 1)}
    for t in (0, 1):
        waves_of[t] = -(-counts[t] // wave_items)
    fft_bytes = 0
    for t in (0, 1):
        nb = algorithmic_bytes(planes[t], n_resp_reads=waves_of[t], items=counts[t])
        fft_bytes += nb["r2c"] + nb["wire"] + nb["c2r"]
    log(f"bench: batched {ms_batch:.2f} ms, sequential {ms_seq:.2f} ms, streams {streams_ms}")
    ach = bins * OPS_PER_BIN / (ms_batch * 1e-3) / 1e9
    return {"workload": "64 events x 3 planes (U, V 800 wires, W 480; 6000 ticks), depos per event "
                        "log-uniform 1e4-1e6 (95% track, 5% points), binomial fluctuation",
            "depos": n_depo, "bins": bins, "reps": reps,
            "depos_per_s": round(n_depo / (ms_batch * 1e-3), 1),
            "plane_frames_per_s": round(len(items) / (ms_batch * 1e-3), 2), "ms_per_batch": round(ms_batch, 3),
            "workspace_bytes": int(nbytes), "workspace_all_items_bytes": int(full),
            "waves": n_waves, "items_per_wave": wave_items,
            "sequential_ms": round(ms_seq, 3), "speedup_vs_sequential": round(ms_seq / ms_batch, 3),
            "streams_ms": streams_ms,
            "fft_algorithmic_bytes": int(fft_bytes),
            "roofline_whole_batch": {"bound": "alu", "achieved": round(ach, 1), "peak": round(VALU_PEAK_GOPS, 1),
                                     "unit": "Gop/s", "frac": round(ach / VALU_PEAK_GOPS, 4),
                                     "note": "bins x ops per bin over the whole batch time (raster and FFT)"}}


# ------------------------------------------------------------------ forward + backward

def leg_fwd_bwd(args, torch, lar, inputs, np):
    from paper_2203_02479_amd.autograd import sim_plane
    log("bench: fwd+bwd, 16 events x 200k depos")
    evs = inputs.cfg4_events()
    P = evs[0].planes[0]
    tune_plane(args, P)
    r = inputs.response_time(P.n_imp, P.half_w, inputs.RESP_TICKS, P.kind)
    resp = lar.spectrum_from_time(P, r).requires_grad_(True)
    deps = [[torch.as_tensor(a).cuda().requires_grad_(True) for a in e.depos[0].arrays()] for e in evs]
    target = torch.zeros((P.n_wires, P.n_ticks), device="cuda")
    n_total = sum(len(e.depos[0]) for e in evs)
    reps = max(10, args.steps // 2)

    def autograd_step():
        for arrs in deps:
            M = sim_plane(*arrs, resp, P, inputs.NSIGMA)
            loss = torch.mean((M - target) ** 2)
            loss.backward()

    ms = med(time_reps(torch, autograd_step, 2, reps))
    # batched plan: forward of all 16 events, the loss gradient, batched backward
    items, off, woff = [], 0, 0
    for e, ev in enumerate(evs):
        n = len(ev.depos[0])
        items.append((0, e, 0, off, n, woff))
        off += n
        woff += P.n_wires * P.n_ticks
    cat = [torch.cat([d[k].detach() for d in deps]) for k in range(5)]
    D = lar.DeviceDepos(*cat)
    wave = torch.empty(woff, device="cuda")
    ws = lar.workspace(min(lar.batch_workspace([P], items, None), BATCH_BUDGET))
    resp_d = resp.detach()
    plan = lar.Batch([P], [resp_d], D, inputs.NSIGMA, None, items, wave, ws, use_graph=True)
    n_waves, wave_items = plan.waves()
    tgt = torch.zeros_like(wave)
    rg = torch.empty_like(resp_d)
    dg = [torch.empty_like(c) for c in cat]
    N = P.n_wires * P.n_ticks

    def batch_step():
        plan.run()
        G = (wave - tgt) * (2.0 / N)                 # d/dM of the per-event MSE
        plan.backward(G, [rg], dg)

    ms_b = med(time_reps(torch, batch_step, 2, reps))
    plan.close()
    log(f"bench: fwd+bwd {ms:.3f} ms (16 autograd steps), batched {ms_b:.3f} ms")
    return {"workload": "16 events x 200k track depos, collection plane 480 x 6000, mean path, MSE loss "
                        "(zero target: the timing does not depend on it)",
            "depos": n_total, "reps": reps,
            "depos_per_s": round(n_total / (ms * 1e-3), 1), "plane_frames_per_s": round(16e3 / ms, 2),
            "ms_per_step": round(ms, 4),
            "batched_ms_per_step": round(ms_b, 4), "batched_depos_per_s": round(n_total / (ms_b * 1e-3), 1),
            "batched_waves": n_waves, "batched_items_per_wave": wave_items,
            "speedup_batched_vs_sequential": round(ms / ms_b, 3)}


# ------------------------------------------------------------------ CPU baseline

def cpu_baseline(P, dep, r, seed, mode, threads):
    import oracle
    oracle.set_threads(threads)
    R = oracle.response_spectrum(P, r)
    t0 = time.perf_counter()
    if mode:
        S = oracle.raster_fluct(P, dep, 3.0, mode=mode, seed=seed, event=0, plane_id=2)
    else:
        S = oracle.raster_mean(P, dep, 3.0)
    oracle.conv_fft(P, S, R)
    t = time.perf_counter() - t0
    oracle.set_threads(1)
    return t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fluct", type=int, default=1, help="0 mean, 1 binomial, 2 Poisson, 3 normal approximation")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-extra", action="store_true", help="headline workload only")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in FFT schedules")
    ap.add_argument("--calib", action="store_true", help="run the copy-kernel counter calibration only")
    ap.add_argument("--atomic-peak", action="store_true",
                    help="time the scattered float-atomic probe only and print its JSON")
    ap.add_argument("--philox-peak", action="store_true",
                    help="time the Philox-block probe (the raster's per-bin draw) and print its JSON")
    ap.add_argument("--copy-floor", action="store_true",
                    help="time the row-copy probe and a flat copy at the time R2C's byte counts and print their JSON")
    ap.add_argument("--leg", choices=["fwd_bwd", "batched", "three_plane"], default=None,
                    help="run only this extra leg and print its JSON (for profiling)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per kernel launch (rocprofv3 FETCH/WRITE_SIZE), if present")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path shards by independent (event, plane) work "
              "items, so a GPU's share is the single-GPU workload.", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        ap.error("--steps must be >= 1")

    import numpy as np
    import torch
    from paper_2203_02479_amd import inputs, lar

    torch.cuda.set_device(0)
    if args.calib:
        copy_calibration(torch)
        return
    if args.atomic_peak:
        print(json.dumps({"atomic_peak": atomic_peak(torch, lar)}), flush=True)
        return
    if args.philox_peak:
        print(json.dumps({"philox_peak": philox_peak(torch, lar)}), flush=True)
        return
    if args.copy_floor:
        print(json.dumps({"copy_floor": copy_floor(torch, lar)}), flush=True)
        return
    legs = {"fwd_bwd": leg_fwd_bwd, "batched": leg_batched, "three_plane": leg_three_plane}
    if args.leg:
        print(json.dumps({args.leg: legs[args.leg](args, torch, lar, inputs, np)}), flush=True)
        return

    log(f"bench: headline, {args.warmup} warm-up + {args.steps} timed steps")
    P, dep, r, seed, steps_ms, per, host_s = leg_forward(args, torch, lar, inputs, np, args.fluct, args.steps,
                                                         args.warmup)
    n_depo = len(dep)
    ms = med(steps_ms)
    log("bench: per-kernel ms (median) " + json.dumps({k: round(v, 4) for k, v in per.items()}))
    traffic = load_traffic(args.traffic)
    nbytes = algorithmic_bytes(P)
    bins = count_bins(P, dep, inputs.NSIGMA)
    fft_roof = fft_roofline(nbytes, per)
    for k in fft_roof:
        fft_roof[k]["traffic"] = traffic.get(k)
    dom = max(per, key=per.get)
    if dom in nbytes:
        roof = {"kernel": dom, "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", **fft_roof[dom]}
    else:
        t_k = per["raster"]
        ach = bins * OPS_PER_BIN / (t_k * 1e-3) / 1e9
        roof = {"kernel": "raster main (k_raster, fluctuated)" if args.fluct else "raster main (k_raster, mean)",
                "bound": "alu", "achieved": round(ach, 1), "peak": round(VALU_PEAK_GOPS, 1), "unit": "Gop/s",
                "frac": round(ach / VALU_PEAK_GOPS, 4), "traffic": traffic.get("raster"),
                "bins": bins, "ops_per_bin": OPS_PER_BIN, "avg_ms": round(t_k, 5)}
    t_all = per["raster"] + per["raster_tail"]
    ach_all = bins * OPS_PER_BIN / (t_all * 1e-3) / 1e9
    roof_raster_all = {"kernels": "k_raster + k_raster_deferred + k_raster_hard + k_raster_flagged",
                       "bound": "alu", "achieved": round(ach_all, 1),
                       "peak": round(VALU_PEAK_GOPS, 1), "unit": "Gop/s", "frac": round(ach_all / VALU_PEAK_GOPS, 4),
                       "avg_ms": round(t_all, 5)}
    # the per-bin draw alone (Philox block + uniform), measured live: the
    # floor of any per-bin counter-based sampler for this event's bins
    pp = philox_peak(torch, lar, reps=10)
    floor_ms = bins / pp["blocks_per_s"] * 1e3
    draw_floor = {"probe": "lar_philox_probe (one Philox4x32-10 block + 52-bit uniform per bin)",
                  "blocks_per_s": round(pp["blocks_per_s"], 1), "bins": bins, "floor_ms": round(floor_ms, 5),
                  "frac_raster_main": round(floor_ms / per["raster"], 4),
                  "frac_raster_all": round(floor_ms / t_all, 4)}
    fft_ms = per["r2c"] + per["wire"] + per["c2r"]
    fft_b = nbytes["r2c"] + nbytes["wire"] + nbytes["c2r"]
    roof_fft_all = {"kernels": "k_r2c_rows + k_wire_static + k_c2r_rows", "bound": "hbm",
                    "achieved": round(fft_b / (fft_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(fft_b / (fft_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "avg_ms": round(fft_ms, 5)}
    mode_name = {0: "mean patches", 1: "binomial fluctuation", 2: "Poisson fluctuation",
                 3: "normal-approximation fluctuation"}
    out = {
        "metric": "depos/s (raster+FFT conv, fwd), 1 MI355X",
        "value": round(n_depo / (ms * 1e-3), 1),
        "unit": "depos/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "ms_per_step_mean": round(statistics.fmean(steps_ms), 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "collection plane 480 wires x 6000 ticks (FFT 512 x 6144), 10 impacts/pitch, "
                               "500k track depos from 60 drift-crossing segments, " + mode_name[args.fluct],
                   "depos": n_depo, "bins": bins, "plane_frames_per_step": 1},
        "plane_frames_per_s": round(1e3 / ms, 2),
        "kernel_ms": {k: round(v, 5) for k, v in per.items()},
        "host_wall_s": round(host_s, 4),
        "roofline": roof,
        "roofline_raster_all": roof_raster_all,
        "raster_draw_floor": draw_floor,
        "roofline_fft_all": roof_fft_all,
        "roofline_fft": fft_roof,
    }
    if not args.skip_extra:
        modes = {}
        for m in (0, 2, 3):
            if m == args.fluct:
                continue
            _, _, _, _, sm, pm, _ = leg_forward(args, torch, lar, inputs, np, m, max(10, args.steps // 2), 2)
            modes[mode_name[m]] = {"ms_per_step": round(med(sm), 5), "depos_per_s": round(n_depo / (med(sm) * 1e-3), 1),
                                   "raster_ms": round(pm["raster"] + pm["raster_tail"], 5)}
            torch.cuda.empty_cache()
        out["modes"] = modes
        for name in ("three_plane", "batched", "fwd_bwd"):
            out[name] = legs[name](args, torch, lar, inputs, np)
            torch.cuda.empty_cache()
    out["fft_schedules"] = dict(TUNED)
    if not args.no_cpu_baseline:
        ncores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        log(f"bench: CPU baseline (FP64 oracle, one full plane-frame) on {ncores} threads and on 1")
        t_n = cpu_baseline(P, dep, r, seed, args.fluct, ncores)
        t_1 = cpu_baseline(P, dep, r, seed, args.fluct, 1)
        sample = (f"one full plane-frame of the headline workload ({n_depo} depos, "
                  f"{mode_name[args.fluct]}): raster + FFT convolution")
        out["cpu_baseline"] = {"value": round(n_depo / t_n, 1), "unit": "depos/s", "cores": ncores, "kind": "oracle",
                               "sample": sample + f", {t_n:.2f} s on {ncores} threads (os.cpu_count() = "
                                         f"{os.cpu_count()})"}
        out["cpu_baseline_1thread"] = {"value": round(n_depo / t_1, 1), "unit": "depos/s", "cores": 1,
                                       "kind": "oracle", "sample": sample + f", {t_1:.2f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
