"""Benchmark: depositions/s of the LArTPC signal-simulation hot path on one
MI355X (raster + scatter-add + FFT convolution).

Headline workload (one step = one plane-frame): the full collection plane,
480 wires x 6000 ticks (time FFT 6144, wire FFT 512), 10 impact positions
per pitch, 500k depositions from 60 seeded cosmic-muon-like segments
crossing a 3.6 m drift, binomial fluctuation on, FP32.  Inputs and the
response spectrum are resident on the device before the timed region.

Also measured (extra fields of the same JSON line):
  fwd_bwd  16 events x 200k depos on the same plane, mean path, forward +
           MSE loss + backward through the autograd wrapper;
  batched  64 events x 3 planes (U, V: 800 wires, W: 480) with log-uniform
           depo counts, one graph-captured batch plan, against 192
           sequential lar_sim_plane calls.

Per-kernel times come from HIP events that the library records on its own
stream between kernels.  The roofline object reports the dominant kernel
against MI355X peaks; the CPU baseline is the FP64 oracle (C raster + numpy
FFT) timed on this host on one full plane-frame.
"""
from __future__ import annotations

import argparse
import json
import os
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(P):
    """HBM bytes each FFT-path kernel must move (read inputs once, write outputs once)."""
    R, N, F = P.n_rows, P.n_ticks, P.nt_fft // 2 + 1
    return {
        "fill": R * N * 4,
        "r2c": R * N * 4 + R * F * 8,
        "wire": R * F * 8 + P.n_imp * P.nw_fft * F * 8 + P.n_wires * F * 8,
        "c2r": P.n_wires * F * 8 + P.n_wires * N * 4,
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


TUNED = {}


def tune_plane(args, P):
    """Time the candidate FFT schedules of this plane shape and register the
    fastest (outside every timed region)."""
    from paper_2203_02479_amd import autotune
    key = autotune.shape_key(P)
    if key in TUNED:
        return
    out = autotune.tune(P, reps=5, cache=False)
    TUNED[key] = {**out["schedule"], "ms": round(out["rows_ms"] + out["wire_ms"], 4),
                  "builtin_ms": round(out["default_ms"], 4), "candidates": out["candidates"]}
    log(f"bench: schedule {key} {json.dumps(TUNED[key])}")


def leg_forward(args, torch, lar, inputs, np):
    log("bench: generating the 500k-depo collection-plane event")
    ev = inputs.cfg1_event()
    P, dep = ev.planes[0], ev.depos[0]
    n_depo = len(dep)
    r = inputs.response_time(P.n_imp, P.half_w, inputs.RESP_TICKS, P.kind)
    D = lar.DeviceDepos.from_host(dep)
    resp = lar.spectrum_from_time(P, r)
    if not args.no_tune:
        tune_plane(args, P)
    seed = inputs.SEED0 + 100
    fl0 = (args.fluct, seed, 0, 2) if args.fluct else None
    ws = lar.workspace(lar.sim_plane_workspace(P, n_depo, fl0))
    wave = torch.empty((P.n_wires, P.n_ticks), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(i):
        fl = (args.fluct, seed, i, 2) if args.fluct else None
        lar.sim_plane(P, D, inputs.NSIGMA, fl, resp, wave, ws, stream)

    log(f"bench: warmup {args.warmup}")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    K = args.steps
    ev_start = torch.cuda.Event(enable_timing=True)
    stage = [[torch.cuda.Event(enable_timing=True) for _ in STAGES] for _ in range(K)]
    for row in stage:                              # materialise the HIP events
        for e in row:
            e.record(stream)
    torch.cuda.synchronize()
    log(f"bench: timing {K} steps")
    t0 = time.perf_counter()
    ev_start.record(stream)
    for i in range(K):
        lar.set_stage_events(stage[i])
        step(args.warmup + i)
    lar.set_stage_events(None)
    torch.cuda.synchronize()
    host_s = time.perf_counter() - t0
    ms = ev_start.elapsed_time(stage[-1][-1]) / K
    per = {n: 0.0 for n in STAGES}
    prev = ev_start
    for i in range(K):
        for s_, n in enumerate(STAGES):
            per[n] += prev.elapsed_time(stage[i][s_])
            prev = stage[i][s_]
    per = {n: v / K for n, v in per.items()}
    log("bench: per-kernel ms " + json.dumps({k: round(v, 4) for k, v in per.items()}))
    return P, dep, r, seed, n_depo, ms, per, host_s


def leg_fwd_bwd(args, torch, lar, inputs, np):
    from paper_2203_02479_amd.autograd import sim_plane
    log("bench: fwd+bwd, 16 events x 200k depos")
    evs = inputs.cfg4_events()
    P = evs[0].planes[0]
    r = inputs.response_time(P.n_imp, P.half_w, inputs.RESP_TICKS, P.kind)
    resp = lar.spectrum_from_time(P, r).requires_grad_(True)
    deps = [[torch.as_tensor(a).cuda().requires_grad_(True) for a in e.depos[0].arrays()] for e in evs]
    target = torch.zeros((P.n_wires, P.n_ticks), device="cuda")
    n_total = sum(len(e.depos[0]) for e in evs)

    def one_step():
        for arrs in deps:
            M = sim_plane(*arrs, resp, P, inputs.NSIGMA)
            loss = torch.mean((M - target) ** 2)
            loss.backward()

    one_step()
    torch.cuda.synchronize()
    K = max(1, args.steps // 5)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(K):
        one_step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / K
    log(f"bench: fwd+bwd {ms:.3f} ms per 16-event step")
    return {"workload": "16 events x 200k track depos, collection plane 480 x 6000, mean path, MSE loss",
            "depos_per_s": round(n_total / (ms * 1e-3), 1), "plane_frames_per_s": round(16e3 / ms, 2),
            "ms_per_step": round(ms, 4), "steps": K}


def leg_batched(args, torch, lar, inputs, np):
    log("bench: batched, 64 events x 3 planes")
    evs = inputs.cfg3_events()
    planes = [evs[0].planes[0], evs[0].planes[2]]              # U/V geometry (type 0), W (type 1)
    resps = [lar.spectrum_from_time(p, inputs.response_time(p.n_imp, p.half_w, inputs.RESP_TICKS, p.kind))
             for p in planes]
    if not args.no_tune:
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
    nbytes = lar.batch_workspace(planes, items, fl)
    log(f"bench: batch workspace {nbytes / 2**30:.1f} GiB")
    ws = lar.workspace(nbytes)
    plan = lar.Batch(planes, resps, D, inputs.NSIGMA, fl, items, wave, ws, use_graph=True)
    plan.run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    R = 3
    a.record()
    for _ in range(R):
        plan.run()
    b.record()
    torch.cuda.synchronize()
    ms_batch = a.elapsed_time(b) / R
    plan.close()
    del ws
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

    seq()
    torch.cuda.synchronize()
    a.record()
    seq()
    b.record()
    torch.cuda.synchronize()
    ms_seq = a.elapsed_time(b)
    n_depo = sum(len(ev.depos[0]) for ev in evs)
    log(f"bench: batched {ms_batch:.2f} ms, sequential {ms_seq:.2f} ms")
    return {"workload": "64 events x 3 planes (U, V 800 wires, W 480; 6000 ticks), depos per event "
                        "log-uniform 1e4-1e6 (95% track, 5% points), binomial fluctuation",
            "depos": n_depo, "depos_per_s": round(n_depo / (ms_batch * 1e-3), 1),
            "plane_frames_per_s": round(len(items) / (ms_batch * 1e-3), 2), "ms_per_batch": round(ms_batch, 3),
            "sequential_ms": round(ms_seq, 3), "speedup_vs_sequential": round(ms_seq / ms_batch, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fluct", type=int, default=1, help="0 mean, 1 binomial, 2 poisson")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-extra", action="store_true", help="headline workload only")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in FFT schedules")
    ap.add_argument("--calib", action="store_true", help="run the copy-kernel counter calibration only")
    ap.add_argument("--leg", choices=["fwd_bwd", "batched"], default=None,
                    help="run only this extra leg and print its JSON (for profiling)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per kernel launch (rocprofv3 FETCH/WRITE_SIZE), if present")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path shards by independent (event, plane) work "
              "items, so a GPU's share is the single-GPU workload.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_02479_amd import inputs, lar

    torch.cuda.set_device(0)
    if args.calib:
        copy_calibration(torch)
        return
    if args.leg:
        leg = leg_fwd_bwd if args.leg == "fwd_bwd" else leg_batched
        print(json.dumps({args.leg: leg(args, torch, lar, inputs, np)}), flush=True)
        return

    P, dep, r, seed, n_depo, ms, per, host_s = leg_forward(args, torch, lar, inputs, np)
    traffic = load_traffic(args.traffic)
    nbytes = algorithmic_bytes(P)
    bins = count_bins(P, dep, inputs.NSIGMA)
    dom = max(per, key=per.get)
    fft_roof = {}
    for k in ("r2c", "wire", "c2r", "fill"):
        ach = nbytes[k] / (per[k] * 1e-3) / 1e9
        fft_roof[k] = {"achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                       "algorithmic_bytes": nbytes[k], "avg_ms": round(per[k], 5), "traffic": traffic.get(k)}
    if dom in nbytes:
        roof = {"kernel": dom, "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", **fft_roof[dom]}
    else:
        t_k = per["raster"]
        ach = bins * OPS_PER_BIN / (t_k * 1e-3) / 1e9
        roof = {"kernel": "raster main (k_raster, fluctuated)" if args.fluct else "raster main (k_raster, mean)",
                "bound": "alu", "achieved": round(ach, 1), "peak": round(VALU_PEAK_GOPS, 1), "unit": "Gop/s",
                "frac": round(ach / VALU_PEAK_GOPS, 4), "traffic": traffic.get("raster"),
                "bins": bins, "ops_per_bin": OPS_PER_BIN, "avg_ms": round(t_k, 5)}
    # the whole raster stage (main kernel + queued draws + flagged
    # sub-chunks) against the same per-bin work: part of the sampling runs after
    # the main kernel
    t_all = per["raster"] + per["raster_tail"]
    ach_all = bins * OPS_PER_BIN / (t_all * 1e-3) / 1e9
    roof_raster_all = {"kernels": "k_raster + k_raster_deferred + k_raster_hard + k_raster_flagged",
                       "bound": "alu", "achieved": round(ach_all, 1),
                       "peak": round(VALU_PEAK_GOPS, 1), "unit": "Gop/s", "frac": round(ach_all / VALU_PEAK_GOPS, 4),
                       "avg_ms": round(t_all, 5)}

    out = {
        "metric": "depos/s (raster+FFT conv, fwd), 1 MI355X",
        "value": round(n_depo / (ms * 1e-3), 1),
        "unit": "depos/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "collection plane 480 wires x 6000 ticks (FFT 512 x 6144), 10 impacts/pitch, "
                               "500k track depos from 60 drift-crossing segments, "
                               + {0: "mean patches", 1: "binomial fluctuation", 2: "Poisson fluctuation"}[args.fluct],
                   "depos": n_depo, "bins": bins, "plane_frames_per_step": 1},
        "plane_frames_per_s": round(1e3 / ms, 2),
        "kernel_ms": {k: round(v, 5) for k, v in per.items()},
        "host_wall_s": round(host_s, 4),
        "roofline": roof,
        "roofline_raster_all": roof_raster_all,
        "roofline_fft": fft_roof,
    }
    if not args.skip_extra:
        out["fwd_bwd"] = leg_fwd_bwd(args, torch, lar, inputs, np)
        torch.cuda.empty_cache()
        out["batched"] = leg_batched(args, torch, lar, inputs, np)
        torch.cuda.empty_cache()

    out["fft_schedules"] = dict(TUNED)
    if not args.no_cpu_baseline:
        import oracle
        log("bench: CPU baseline (FP64 oracle, one full plane-frame, one thread)")
        R = oracle.response_spectrum(P, r)
        t0 = time.perf_counter()
        if args.fluct:
            S = oracle.raster_fluct(P, dep, inputs.NSIGMA, mode=args.fluct, seed=seed, event=0, plane_id=2)
        else:
            S = oracle.raster_mean(P, dep, inputs.NSIGMA)
        oracle.conv_fft(P, S, R)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(n_depo / t_cpu, 1), "unit": "depos/s", "cores": 1, "kind": "oracle",
                               "sample": f"one full plane-frame ({n_depo} depos) of the headline workload, "
                                         f"{t_cpu:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
