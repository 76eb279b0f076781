"""Seeded synthetic inputs: plane geometry, drifted depositions, detector responses.

This module only *generates inputs*.  It holds none of the simulation's
arithmetic (no binning, no sampling, no Fourier transforms) and it is the one
module shared by the FP64 oracle tests and the GPU path.  Every array is
generated in float64 with ``numpy.random.Generator(PCG64(seed))`` and rounded
once to float32, which is what both sides consume.

Physics of the inputs (the drift stage itself is upstream of the simulated
path, paper Sec. 2.2: ionization groups are diffused while drifting):

* drift velocity 1.6 mm/us, longitudinal diffusion D_L = 4 cm^2/s,
  transverse D_T = 8.8 cm^2/s;
* sigma_L [us] = sqrt(2 D_L t) / v and sigma_T [mm] = sqrt(2 D_T t) for a
  group that drifted for t microseconds;
* tracks are straight segments sampled at fixed steps (the paper's inputs are
  ionization groups sampled along charged-particle steps, Sec. 2.2), with a
  constant charge per mm; isolated point depositions carry log-uniform charge.

Units: time in microseconds, lengths in mm, charge in electrons.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

D_L = 4.0e-4        # mm^2/us  (4 cm^2/s)
D_T = 8.8e-4        # mm^2/us  (8.8 cm^2/s)
V_DRIFT = 1.6       # mm/us
PITCH = 5.0         # mm
TICK = 0.5          # us
N_IMP = 10          # impact positions per pitch
HALF_W = 10         # response half-width in wires (21 wires)
RESP_TICKS = 200    # response length in ticks
Q_PER_MM = 5000.0   # electrons per mm of track
NSIGMA = 3.0
SEED0 = 20220305

SIN60 = math.sin(math.radians(60.0))
COS60 = 0.5
LIFETIME = 10000.0  # us, electron lifetime of the drift-stage inputs (10 ms)
# pitch coordinate of each plane kind as (cos, sin, offset): x = z cos + y sin + offset
PLANE_PROJ = {"U": (COS60, SIN60, 0.0), "V": (COS60, -SIN60, 3000.0 * SIN60), "W": (1.0, 0.0, 0.0)}


def smooth_length(n: int, even: bool = False) -> int:
    """Smallest 2^a * 3^b >= n (optionally also even)."""
    best = None
    p2 = 1
    while p2 < 4 * max(n, 1):
        v = p2
        while v < 4 * max(n, 1):
            if v >= n and (not even or v % 2 == 0):
                if best is None or v < best:
                    best = v
            v *= 3
        p2 *= 2
    return best


@dataclass
class Plane:
    """Geometry of one wire plane (paper Sec. 2.1: each plane is simulated on
    its own 2D drift-time x wire-pitch space)."""
    n_wires: int
    n_ticks: int
    n_imp: int = N_IMP
    nt_fft: int = 0
    nw_fft: int = 0
    pitch: float = PITCH
    x0: float = PITCH / 2.0      # centre of wire 0, so impact row 0 starts at 0 mm
    tick: float = TICK
    t0: float = 0.0
    kind: str = "unipolar"       # response shape (collection = unipolar)
    half_w: int = HALF_W

    def __post_init__(self):
        if self.nt_fft == 0:
            self.nt_fft = smooth_length(self.n_ticks, even=True)
        if self.nw_fft == 0:
            self.nw_fft = smooth_length(self.n_wires + 2 * self.half_w)

    @property
    def n_rows(self) -> int:
        return self.n_wires * self.n_imp

    @property
    def n_freq(self) -> int:
        return self.nt_fft // 2 + 1


@dataclass
class Depos:
    """Structure of arrays of drifted depositions for one plane (float32)."""
    q: np.ndarray
    t: np.ndarray
    x: np.ndarray
    sigma_t: np.ndarray
    sigma_x: np.ndarray

    def __len__(self):
        return int(self.q.shape[0])

    def arrays(self):
        return (self.q, self.t, self.x, self.sigma_t, self.sigma_x)

    def take(self, idx) -> "Depos":
        return Depos(*(a[idx] for a in self.arrays()))


@dataclass
class Event:
    """One event: 3D points shared by all planes and per-plane depositions."""
    planes: list
    depos: list
    seed: int
    meta: dict = field(default_factory=dict)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def diffuse(xd):
    """Drift time and diffusion widths for drift distances xd (mm), float64."""
    t = xd / V_DRIFT
    sl = np.sqrt(2.0 * D_L * t) / V_DRIFT
    st = np.sqrt(2.0 * D_T * t)
    return t, sl, st


def pitch_coord(kind: str, y, z):
    """Transverse (pitch) coordinate of a 3D point for the U, V, W planes."""
    if kind == "W":
        return z
    if kind == "U":
        return z * COS60 + y * SIN60
    if kind == "V":
        return z * COS60 - y * SIN60 + 3000.0 * SIN60
    raise ValueError(kind)


def _points_along(A, B, s):
    """Points at arc lengths s (mm) from A toward B."""
    d = B - A
    L = np.linalg.norm(d)
    return A[None, :] + (s / L)[:, None] * d[None, :]


def crossing_segments(rng, n_seg, drift=3600.0, ymax=3000.0, zmax=2400.0):
    """Cosmic-muon-like segments crossing the full drift: A=(0,ya,za), B=(drift,yb,zb)."""
    A = np.stack([np.zeros(n_seg), rng.uniform(0, ymax, n_seg), rng.uniform(0, zmax, n_seg)], 1)
    B = np.stack([np.full(n_seg, drift), rng.uniform(0, ymax, n_seg), rng.uniform(0, zmax, n_seg)], 1)
    return A, B


def even_track_points(A, B, n_total):
    """n_total points evenly spaced (step h = total length / n_total) along the
    concatenated segments; returns (points [n,3], h)."""
    L = np.linalg.norm(B - A, axis=1)
    h = L.sum() / n_total
    s_all = (np.arange(n_total) + 0.5) * h
    cum = np.concatenate([[0.0], np.cumsum(L)])
    seg = np.clip(np.searchsorted(cum, s_all, side="right") - 1, 0, len(L) - 1)
    pts = np.empty((n_total, 3))
    for i in range(len(L)):
        sel = seg == i
        if sel.any():
            pts[sel] = _points_along(A[i], B[i], s_all[sel] - cum[i])
    return pts, h


def _to_depos(pts, q, kind):
    t, sl, st = diffuse(pts[:, 0])
    x = pitch_coord(kind, pts[:, 1], pts[:, 2])
    f = np.float32
    return Depos(q.astype(f), t.astype(f), x.astype(f), sl.astype(f), st.astype(f))


# ----------------------------------------------------------------- configs

def cfg0_plane() -> Plane:
    return Plane(n_wires=64, n_ticks=1024, kind="unipolar")


def cfg0_event(seed=SEED0 + 0) -> Event:
    """4 straight tracks in a 800 x 1000 x 320 mm box (drift, y, z), 500 depos
    each at 1 mm steps, 5000 e-/mm, on one 64-wire collection plane."""
    rng = _rng(seed)
    pts = []
    for _ in range(4):
        while True:
            A = np.array([rng.uniform(0, 800), rng.uniform(0, 1000), rng.uniform(0, 320)])
            B = np.array([rng.uniform(0, 800), rng.uniform(0, 1000), rng.uniform(0, 320)])
            if np.linalg.norm(B - A) >= 500.0:
                break
        pts.append(_points_along(A, B, np.arange(500) + 0.5))
    pts = np.concatenate(pts)
    q = np.full(len(pts), Q_PER_MM * 1.0)
    return Event([cfg0_plane()], [_to_depos(pts, q, "W")], seed)


def cfg1_plane() -> Plane:
    return Plane(n_wires=480, n_ticks=6000, kind="unipolar")


def track_event(seed, n_seg, n_depo, planes_kinds, n_points=0):
    rng = _rng(seed)
    A, B = crossing_segments(rng, n_seg)
    pts, h = even_track_points(A, B, n_depo)
    q = np.full(n_depo, Q_PER_MM * h)
    if n_points:
        P = np.stack([rng.uniform(0, 3600, n_points), rng.uniform(0, 3000, n_points),
                      rng.uniform(0, 2400, n_points)], 1)
        qp = 10.0 ** rng.uniform(2.0, 5.0, n_points)
        pts = np.concatenate([pts, P])
        q = np.concatenate([q, qp])
    return pts, q, h


def cfg1_event(seed=SEED0 + 100, n_depo=500_000, n_seg=60) -> Event:
    """60 crossing segments, n_depo depos evenly spaced, collection plane."""
    pts, q, h = track_event(seed, n_seg, n_depo, ["W"])
    return Event([cfg1_plane()], [_to_depos(pts, q, "W")], seed, {"step_mm": h})


def cfg2_planes():
    return [Plane(n_wires=800, n_ticks=6000, kind="bipolar"),
            Plane(n_wires=800, n_ticks=6000, kind="bipolar"),
            Plane(n_wires=480, n_ticks=6000, kind="unipolar")]


def cfg2_event(seed=SEED0 + 200, n_track=1_900_000, n_points=100_000, n_seg=228) -> Event:
    pts, q, h = track_event(seed, n_seg, n_track, None, n_points)
    depos = [_to_depos(pts, q, k) for k in ("U", "V", "W")]
    return Event(cfg2_planes(), depos, seed, {"step_mm": h})


def cfg3_events(n_events=64, seed0=SEED0 + 300):
    """Per-event depo counts log-uniform in 1e4..1e6; 95% track, 5% points."""
    evs = []
    for e in range(n_events):
        seed = seed0 + e
        rng = _rng(seed)
        n_e = int(np.rint(10.0 ** rng.uniform(4.0, 6.0)))
        n_pt = n_e - int(np.rint(0.95 * n_e))
        n_tr = n_e - n_pt
        n_seg = int(math.ceil(n_tr / 8333.0))
        evs.append(cfg2_event(seed=seed + 1_000_000, n_track=n_tr, n_points=n_pt, n_seg=n_seg))
    return evs


def cfg4_events(n_events=16, n_depo=200_000, seed0=SEED0 + 400):
    return [cfg1_event(seed=seed0 + e, n_depo=n_depo, n_seg=24) for e in range(n_events)]


def undrifted_groups(seed, n_seg, n_depo, n_points=0):
    """Ionization groups before the drift stage, as float32 arrays
    (q0, t0, xd, y, z): the tracks (and isolated points) of track_event, with
    xd the distance to the anode along the drift and t0 = 0 (event time)."""
    pts, q, _ = track_event(seed, n_seg, n_depo, None, n_points)
    f = np.float32
    return (q.astype(f), np.zeros(len(q), f), pts[:, 0].astype(f), pts[:, 1].astype(f),
            pts[:, 2].astype(f))


def noise_amplitude(plane, rms=200.0, rise=2.0, corner=0.02):
    """Synthetic noise amplitude per frequency bin f <= nt_fft/2 (float32, in
    waveform units): a flat floor that gives about `rms` per tick, times a
    low-frequency rise 1 + rise * exp(-f / (corner * F))."""
    F = plane.nt_fft // 2 + 1
    f = np.arange(F, dtype=np.float64)
    floor = rms * math.sqrt(plane.nt_fft / 2.0)
    return (floor * (1.0 + rise * np.exp(-f / (corner * F)))).astype(np.float32)


# --------------------------------------------------------------- responses

def response_time(n_imp=N_IMP, half_w=HALF_W, n_rt=RESP_TICKS, kind="unipolar"):
    """Synthetic field x electronics response r[k][dw + half_w][tau] (float32).

    Gaussian-in-time (unipolar, collection) or derivative-of-Gaussian
    (bipolar, induction) shape centred at tick 100 with width 20 ticks, times
    exp(-|dw - o_k| / 1.5) across wires, where o_k = (k + 1/2)/n_imp - 1/2 is
    the impact offset of sub-row k in pitches.  Causal in time."""
    tau = np.arange(n_rt, dtype=np.float64)
    u = (tau - 100.0) / 20.0
    g = np.exp(-0.5 * u * u)
    if kind == "bipolar":
        g = -u * g
    dw = np.arange(-half_w, half_w + 1, dtype=np.float64)
    ok = (np.arange(n_imp) + 0.5) / n_imp - 0.5
    sp = np.exp(-np.abs(dw[None, :] - ok[:, None]) / 1.5)
    r = sp[:, :, None] * g[None, None, :]
    return r.astype(np.float32)


def random_spectrum(plane: Plane, seed: int, scale=1.0):
    """Arbitrary complex spectrum [n_imp][nw_fft][nt_fft/2+1] as interleaved
    float32 (re, im) pairs: a generic input for the convolution operator."""
    rng = _rng(seed)
    shape = (plane.n_imp, plane.nw_fft, plane.n_freq, 2)
    return (scale * rng.standard_normal(shape)).astype(np.float32)


def random_grid(plane: Plane, seed: int, density=1.0):
    rng = _rng(seed)
    g = rng.standard_normal((plane.n_rows, plane.n_ticks))
    if density < 1.0:
        g *= rng.uniform(size=g.shape) < density
    return g.astype(np.float32)


def random_depos(plane: Plane, n: int, seed: int, sigma_scale=1.0, margin=0.0):
    """Uniformly scattered depositions over the plane (plus optional margin
    outside it, to exercise clipping)."""
    rng = _rng(seed)
    T = plane.n_ticks * plane.tick
    X = plane.n_rows * plane.pitch / plane.n_imp
    x_lo = plane.x0 - plane.pitch / 2.0
    t = rng.uniform(plane.t0 - margin * T, plane.t0 + (1 + margin) * T, n)
    x = rng.uniform(x_lo - margin * X, x_lo + (1 + margin) * X, n)
    st = sigma_scale * rng.uniform(0.2, 1.5, n) * plane.tick
    sx = sigma_scale * rng.uniform(0.2, 4.0, n) * plane.pitch / plane.n_imp
    q = rng.uniform(100.0, 5000.0, n)
    f = np.float32
    return Depos(q.astype(f), t.astype(f), x.astype(f), st.astype(f), sx.astype(f))
