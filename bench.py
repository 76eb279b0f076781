"""Benchmark: depositions/s of the LArTPC signal-simulation hot path on one
MI355X (raster + scatter-add + FFT convolution, one plane-frame per step).

Workload (default): the full collection plane -- 480 wires x 6000 ticks
(time FFT 6144, wire FFT 512), 10 impact positions per pitch, 500k
depositions from 60 seeded cosmic-muon-like segments crossing a 3.6 m
drift, binomial fluctuation on, FP32.  Inputs and the response spectrum are
resident on the device before the timed region.

Prints one JSON line (rank 0).  Per-kernel times come from HIP events that
the library records on its own stream between kernels; the roofline object
reports the dominant kernel against MI355X peaks.  The CPU baseline is the
FP64 oracle (C raster + numpy FFT) timed on this host on a bounded sample.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(P):
    """HBM bytes each kernel must move at minimum (read inputs once, write outputs once)."""
    R, N, F = P.n_rows, P.n_ticks, P.nt_fft // 2 + 1
    return {
        "fill": R * N * 4,
        "r2c": R * N * 4 + R * F * 8,
        "wire": R * F * 8 + P.n_imp * P.nw_fft * F * 8 + P.n_wires * F * 8,
        "c2r": P.n_wires * F * 8 + P.n_wires * N * 4,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fluct", type=int, default=1, help="0 mean, 1 binomial, 2 poisson")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per kernel (rocprofv3 FETCH/WRITE_SIZE), if present")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path shards by independent (event, plane) work "
              "items and this build measures a single GPU's share.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_02479_amd import inputs, lar

    torch.cuda.set_device(0)
    log("bench: generating the 500k-depo collection-plane event")
    ev = inputs.cfg1_event()
    P, dep = ev.planes[0], ev.depos[0]
    n_depo = len(dep)
    r = inputs.response_time(P.n_imp, P.half_w, inputs.RESP_TICKS, P.kind)
    D = lar.DeviceDepos.from_host(dep)
    resp = lar.spectrum_from_time(P, r)
    seed = inputs.SEED0 + 100
    ws = lar.workspace(lar.sim_plane_workspace(P, n_depo, (args.fluct, seed, 0, 2) if args.fluct else None))
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
    stage = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    for row in stage:            # materialise the HIP events
        for e in row:
            e.record(stream)
    ev_start.record(stream)
    torch.cuda.synchronize()

    log(f"bench: timing {K} steps")
    t_host0 = time.perf_counter()
    ev_start.record(stream)
    for i in range(K):
        lar.set_stage_events(stage[i])
        step(args.warmup + i)
    lar.set_stage_events(None)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host0
    total_ms = ev_start.elapsed_time(stage[-1][4])
    ms = total_ms / K
    names = ["fill", "raster", "r2c", "wire", "c2r"]
    per = {n: 0.0 for n in names}
    prev = ev_start
    for i in range(K):
        for s, n in enumerate(names):
            per[n] += prev.elapsed_time(stage[i][s])
            prev = stage[i][s]
    per = {n: v / K for n, v in per.items()}
    log("bench: per-kernel ms " + json.dumps({k: round(v, 4) for k, v in per.items()}))

    # roofline of the dominant kernel
    nbytes = algorithmic_bytes(P)
    dom = max(per, key=per.get)
    traffic = None
    if os.path.exists(args.traffic):
        try:
            tr = json.load(open(args.traffic))
            traffic = tr.get(dom)
        except Exception:
            traffic = None
    if dom in nbytes:
        ach = nbytes[dom] / (per[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes": nbytes[dom], "avg_ms": round(per[dom], 5)}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": traffic, "avg_ms": round(per[dom], 5)}

    out = {
        "metric": "depos/s (raster+FFT conv, fwd), 1 MI355X",
        "value": round(n_depo / (ms * 1e-3), 1),
        "unit": "depos/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "collection plane 480 wires x 6000 ticks (FFT 512 x 6144), 10 impacts/pitch, "
                               "500k track depos, binomial fluctuation" if args.fluct == 1 else
                               "collection plane 480 x 6000, 500k track depos, fluctuation mode %d" % args.fluct,
                   "depos": n_depo, "plane_frames_per_step": 1, "fluct": args.fluct},
        "plane_frames_per_s": round(1e3 / ms, 2),
        "kernel_ms": {k: round(v, 5) for k, v in per.items()},
        "host_wall_s": round(t_host, 4),
        "roofline": roof,
    }

    if not args.no_cpu_baseline:
        import oracle
        log("bench: CPU baseline (FP64 oracle, one full plane-frame)")
        R = oracle.response_spectrum(P, r)
        t0 = time.perf_counter()
        if args.fluct:
            S = oracle.raster_fluct(P, dep, inputs.NSIGMA, mode=args.fluct, seed=seed, event=0, plane_id=2)
        else:
            S = oracle.raster_mean(P, dep, inputs.NSIGMA)
        oracle.conv_fft(P, S, R)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(n_depo / t_cpu, 1), "unit": "depos/s", "cores": 1, "kind": "oracle",
                               "sample": f"one full plane-frame ({n_depo} depos), {t_cpu:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
