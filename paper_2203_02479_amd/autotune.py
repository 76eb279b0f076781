"""Timing-based choice of FFT-convolution and raster launch schedules, with a
JSON cache.

For one plane shape, every candidate schedule of the C library
(``lar_schedule_candidates``) runs ``lar_fftconv`` on the same synthetic
grid and response; HIP events recorded after each stage give the time of
the two time-axis row passes (real FFT + inverse real FFT) and of the fused
wire pass.  Row and wire choices are independent (the stages share only
the spectrum buffers), so the best row choice and the best wire choice are
combined and registered with ``lar_schedule_set``.  A candidate whose
waveforms differ from the built-in schedule's by more than float rounding
(relative L2 above 1e-5) is rejected.

The raster's per-wave LDS tile (``raster_tile``) is chosen apart by
``tune_raster``, on the caller's depositions: which size is fastest depends
on how many sub-chunks' bounding boxes fit it, so on the depo widths and
spacing as well as on the shape.  Every tile gives the same fluctuated
counts (bit for bit) and the same mean patches up to float rounding; a tile
whose grid differs from the built-in tile's beyond that is rejected.

The cache maps ``arch -> shape key -> schedule`` and lives at
``$LAR_TUNE_CACHE`` or ``~/.cache/lar_sim/schedules.json``.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import lar

ROW_KEYS = ("row_threads", "row_order")
WIRE_KEYS = ("wire_cols", "wire_threads", "wire_order")
FFT_KEYS = ROW_KEYS + WIRE_KEYS


def cache_path() -> str:
    return os.environ.get("LAR_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "lar_sim", "schedules.json")


def shape_key(plane) -> str:
    return f"{plane.n_wires}x{plane.n_imp}x{plane.n_ticks}/{plane.nt_fft}x{plane.nw_fft}"


def device_arch(device="cuda") -> str:
    props = torch.cuda.get_device_properties(torch.device(device))
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _read(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _write(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _stage_times(plane, grid, resp, wave, ws, reps, stream):
    """Median (rows ms, wire ms) over reps runs of lar_fftconv."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    start = torch.cuda.Event(enable_timing=True)
    for e in ev:                  # torch creates the HIP event on its first record
        e.record(stream)
    rows, wire = [], []
    lar.set_stage_events(ev)
    try:
        for _ in range(reps):
            start.record(stream)
            lar.fftconv(plane, grid, resp, wave, ws, stream)
            stream.synchronize()
            r2c = start.elapsed_time(ev[3])
            w = ev[3].elapsed_time(ev[4])
            c2r = ev[4].elapsed_time(ev[5])
            rows.append(r2c + c2r)
            wire.append(w)
    finally:
        lar.set_stage_events(None)
    return statistics.median(rows), statistics.median(wire)


def tune(plane, device="cuda", reps=10, warmup=2, seed=1234, apply=True, cache=True, verbose=False) -> dict:
    """Time every candidate schedule of this plane shape and return
    {"schedule": best, "rows_ms": ..., "wire_ms": ..., "default_ms": ...}.
    With apply, the best schedule is registered; with cache, it is stored
    under this device's arch."""
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    R = plane.n_wires * plane.n_imp
    grid = torch.rand((R, plane.n_ticks), generator=gen, dtype=torch.float32).to(dev)
    resp = torch.randn((plane.n_imp, plane.nw_fft, plane.nt_fft // 2 + 1, 2), generator=gen,
                       dtype=torch.float32).to(dev)
    wave = torch.empty((plane.n_wires, plane.n_ticks), dtype=torch.float32, device=dev)
    ws = lar.workspace(lar.fftconv_workspace(plane), dev)

    previous = lar.schedule_get(plane)
    default = lar.schedule_default(plane)
    results = []
    ref = None
    try:
        for cand in lar.schedule_candidates(plane):
            if cand["raster_tile"] != default["raster_tile"]:   # raster choices: tune_raster
                continue
            lar.schedule_set(plane, cand)
            for _ in range(warmup):
                lar.fftconv(plane, grid, resp, wave, ws, stream)
            stream.synchronize()
            if ref is None:           # the first candidate is the built-in schedule
                ref = wave.clone()
                ref_norm = float(torch.linalg.vector_norm(ref))
            err = float(torch.linalg.vector_norm(wave - ref)) / max(ref_norm, 1e-30)
            if err > 1e-5:
                if verbose:
                    print(f"[autotune] {shape_key(plane)} rejects {cand}: rel err {err:.2e}", flush=True)
                continue
            rows_ms, wire_ms = _stage_times(plane, grid, resp, wave, ws, reps, stream)
            results.append((cand, rows_ms, wire_ms))
    finally:
        lar.schedule_set(plane, previous if previous != default else None)
    if not results:
        raise RuntimeError(f"no schedule of {shape_key(plane)} passed the output check")

    def same(a, b, keys):
        return all(a[k] == b[k] for k in keys)

    # rows: candidates that keep the built-in wire pass; wire: those that keep the built-in rows
    row_c = [r for r in results if same(r[0], default, WIRE_KEYS)]
    wire_c = [r for r in results if same(r[0], default, ROW_KEYS)]
    best_row = min(row_c, key=lambda r: r[1])
    best_wire = min(wire_c, key=lambda r: r[2])
    best = dict(previous)         # keeps a raster tile tuned before
    best.update({k: best_row[0][k] for k in ROW_KEYS})
    best.update({k: best_wire[0][k] for k in WIRE_KEYS})
    d_row = next(r for r in results if r[0] == default)
    out = {"schedule": best, "rows_ms": best_row[1], "wire_ms": best_wire[2],
           "default_ms": d_row[1] + d_row[2], "candidates": len(results)}
    if verbose:
        print(f"[autotune] {shape_key(plane)}: {best} rows {best_row[1]:.4f} ms wire {best_wire[2]:.4f} ms "
              f"(built-in {out['default_ms']:.4f} ms, {len(results)} candidates)", flush=True)
    if apply:
        lar.schedule_set(plane, best)
    if cache:
        path = cache_path()
        data = _read(path)
        data.setdefault(device_arch(dev), {})[shape_key(plane)] = {
            "schedule": best, "ms": best_row[1] + best_wire[2]}
        _write(path, data)
    return out


def tune_raster(plane, depos, nsigma, fluct, device="cuda", reps=5, warmup=2, apply=True, cache=True,
                verbose=False) -> dict:
    """Time lar_raster over these device depositions (lar.DeviceDepos) for
    every raster tile of this plane shape's candidates, the FFT choices
    held at the schedule in effect, and return {"raster_tile": best,
    "ms": {tile: median ms}}.  With apply, the best tile is registered;
    with cache, stored with the shape's schedule under this device's arch."""
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev)
    current = lar.schedule_get(plane)
    default = lar.schedule_default(plane)
    tiles = sorted({c["raster_tile"] for c in lar.schedule_candidates(plane)})
    grid = torch.zeros((plane.n_wires * plane.n_imp, plane.n_ticks), dtype=torch.float32, device=dev)
    ws = lar.workspace(lar.raster_workspace(plane, len(depos), fluct), dev)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times, ref = {}, None
    try:
        for tile in [default["raster_tile"]] + [t for t in tiles if t != default["raster_tile"]]:
            lar.schedule_set(plane, dict(current, raster_tile=tile))
            samples = []
            for i in range(warmup + reps):
                grid.zero_()
                start.record(stream)
                lar.raster(plane, depos, nsigma, fluct, grid, ws, stream)
                end.record(stream)
                stream.synchronize()
                if i >= warmup:
                    samples.append(start.elapsed_time(end))
            if ref is None:           # the built-in tile first
                ref = grid.clone()
                ref_norm = max(float(torch.linalg.vector_norm(ref)), 1e-30)
            else:
                exact = fluct is not None and fluct[0] != 0
                err = float(torch.linalg.vector_norm(grid - ref)) / ref_norm
                if (exact and not torch.equal(grid, ref)) or err > 1e-6:
                    if verbose:
                        print(f"[autotune] {shape_key(plane)} rejects raster tile {tile}: rel err {err:.2e}",
                              flush=True)
                    continue
            times[tile] = statistics.median(samples)
    finally:
        lar.schedule_set(plane, current if current != default else None)
    best = min(times, key=times.get)
    if verbose:
        print(f"[autotune] {shape_key(plane)} raster tiles {times} -> {best}", flush=True)
    if apply:
        lar.schedule_set(plane, dict(current, raster_tile=best))
    if cache:
        path = cache_path()
        data = _read(path)
        entry = data.setdefault(device_arch(dev), {}).setdefault(shape_key(plane), {"schedule": current})
        entry["schedule"] = dict(entry["schedule"], raster_tile=best)
        _write(path, data)
    return {"raster_tile": best, "ms": times}


def load(planes, device="cuda", path=None) -> int:
    """Register the cached schedules of these plane shapes for this
    device's arch; returns how many were found."""
    data = _read(path or cache_path()).get(device_arch(device), {})
    n = 0
    for p in planes:
        entry = data.get(shape_key(p))
        if entry:
            lar.schedule_set(p, entry["schedule"])
            n += 1
    return n


def ensure(planes, device="cuda", reps=10, verbose=False) -> dict:
    """Cached schedule for each shape, tuning the shapes not in the cache."""
    out = {}
    seen = set()
    data = _read(cache_path()).get(device_arch(device), {})
    for p in planes:
        k = shape_key(p)
        if k in seen:
            continue
        seen.add(k)
        if k in data:
            lar.schedule_set(p, data[k]["schedule"])
            out[k] = data[k]["schedule"]
        else:
            out[k] = tune(p, device=device, reps=reps, verbose=verbose)["schedule"]
    return out
