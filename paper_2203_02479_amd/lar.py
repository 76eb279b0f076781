"""ctypes binding of the gfx950 library ``liblar.so`` (C ABI in include/lar.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Arrays are torch tensors on the GPU (device
pointers are passed through); the stream is the caller's current HIP stream
unless one is given.  There is no CPU fallback: if the library is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblar.so")

LAR_OK, LAR_EINVAL, LAR_ESIZE, LAR_EWORKSPACE, LAR_EHIP = 0, -1, -2, -3, -4


class LarError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {_lib().lar_status_str(status).decode()} (status {status}"
                         + (f", hip error {_lib().lar_last_hip_error()})" if status == LAR_EHIP else ")"))


class lar_plane(ctypes.Structure):
    _fields_ = [("n_wires", ctypes.c_int32), ("n_imp", ctypes.c_int32), ("n_ticks", ctypes.c_int32),
                ("nt_fft", ctypes.c_int32), ("nw_fft", ctypes.c_int32), ("pitch", ctypes.c_float),
                ("x0", ctypes.c_float), ("tick", ctypes.c_float), ("t0", ctypes.c_float)]


class lar_depos(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p), ("t", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("sigma_t", ctypes.c_void_p), ("sigma_x", ctypes.c_void_p), ("n", ctypes.c_int64)]


class lar_fluct(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("event", ctypes.c_uint32), ("plane", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class lar_batch_item(ctypes.Structure):
    _fields_ = [("plane_type", ctypes.c_int32), ("event", ctypes.c_uint32), ("plane", ctypes.c_uint32),
                ("reserved", ctypes.c_int32), ("depo_offset", ctypes.c_int64), ("n_depos", ctypes.c_int64),
                ("wave_offset", ctypes.c_int64)]


class lar_drift_params(ctypes.Structure):
    _fields_ = [("speed", ctypes.c_float), ("diff_l", ctypes.c_float), ("diff_t", ctypes.c_float),
                ("lifetime", ctypes.c_float)]


class lar_plane_proj(ctypes.Structure):
    _fields_ = [("cos_a", ctypes.c_float), ("sin_a", ctypes.c_float), ("offset", ctypes.c_float)]


class lar_schedule(ctypes.Structure):
    _fields_ = [("row_threads", ctypes.c_int32), ("row_order", ctypes.c_int32), ("wire_cols", ctypes.c_int32),
                ("wire_threads", ctypes.c_int32), ("wire_order", ctypes.c_int32), ("raster_tile", ctypes.c_int32)]

    FIELDS = ("row_threads", "row_order", "wire_cols", "wire_threads", "wire_order", "raster_tile")

    def as_dict(self):
        return {k: int(getattr(self, k)) for k in self.FIELDS}


# name -> (argtypes, restype); every symbol declared in include/lar.h
_P, _VP, _SZ = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t
SIGNATURES = {
    "lar_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "lar_last_hip_error": ([], ctypes.c_int),
    "lar_raster_workspace": ([_P(lar_plane), ctypes.c_int64, _P(lar_fluct), _P(_SZ)], ctypes.c_int),
    "lar_raster": ([_P(lar_plane), _P(lar_depos), ctypes.c_float, _P(lar_fluct), _VP, _VP, _SZ, _VP],
                   ctypes.c_int),
    "lar_fftconv_workspace": ([_P(lar_plane), _P(_SZ)], ctypes.c_int),
    "lar_fftconv": ([_P(lar_plane), _VP, _VP, _VP, _VP, _SZ, _VP], ctypes.c_int),
    "lar_fftconv_noalloc_max_bytes": ([], ctypes.c_size_t),
    "lar_fftconv_noalloc": ([_P(lar_plane), _VP, _VP, _VP, _VP], ctypes.c_int),
    "lar_sim_plane_workspace": ([_P(lar_plane), ctypes.c_int64, _P(lar_fluct), _P(_SZ)], ctypes.c_int),
    "lar_sim_plane": ([_P(lar_plane), _P(lar_depos), ctypes.c_float, _P(lar_fluct), _VP, _VP, _VP, _SZ,
                       _VP], ctypes.c_int),
    "lar_response_spectrum_workspace": ([_P(lar_plane), ctypes.c_int32, ctypes.c_int32, _P(_SZ)],
                                        ctypes.c_int),
    "lar_response_spectrum": ([_P(lar_plane), _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _SZ, _VP],
                              ctypes.c_int),
    "lar_fftconv_backward_workspace": ([_P(lar_plane), _P(_SZ)], ctypes.c_int),
    "lar_fftconv_backward": ([_P(lar_plane), _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP], ctypes.c_int),
    "lar_fftconv_backward_spec_workspace": ([_P(lar_plane), _P(_SZ)], ctypes.c_int),
    "lar_fftconv_backward_spec": ([_P(lar_plane), _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _SZ, _VP],
                                  ctypes.c_int),
    "lar_raster_backward": ([_P(lar_plane), _P(lar_depos), ctypes.c_float, _VP, _VP, _VP, _VP, _VP, _VP, _VP],
                            ctypes.c_int),
    "lar_batch_workspace": ([_P(lar_plane), ctypes.c_int32, _P(lar_batch_item), ctypes.c_int32, _P(lar_fluct),
                             _P(_SZ)], ctypes.c_int),
    "lar_batch_create": ([_P(lar_plane), ctypes.c_int32, _P(_VP), _P(lar_depos), ctypes.c_float, _P(lar_fluct),
                          _P(lar_batch_item), ctypes.c_int32, _VP, _VP, _SZ, ctypes.c_int32, _P(_VP)], ctypes.c_int),
    "lar_batch_workspace_waves": ([_P(lar_plane), ctypes.c_int32, _P(lar_batch_item), ctypes.c_int32,
                                   _P(lar_fluct), ctypes.c_int32, _P(_SZ)], ctypes.c_int),
    "lar_batch_waves": ([_VP, _P(ctypes.c_int32), _P(ctypes.c_int32)], ctypes.c_int),
    "lar_batch_backward": ([_VP, _VP, _P(_VP), _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "lar_batch_run": ([_VP, _VP], ctypes.c_int),
    "lar_sim_streams_workspace": ([_P(lar_plane), ctypes.c_int32, _P(lar_batch_item), ctypes.c_int32,
                                   _P(lar_fluct), ctypes.c_int32, _P(_SZ)], ctypes.c_int),
    "lar_sim_streams": ([_P(lar_plane), ctypes.c_int32, _P(_VP), _P(lar_depos), ctypes.c_float, _P(lar_fluct),
                         _P(lar_batch_item), ctypes.c_int32, _VP, _P(_VP), ctypes.c_int32, _VP, _SZ, _VP],
                        ctypes.c_int),
    "lar_batch_destroy": ([_VP], ctypes.c_int),
    "lar_set_stage_events": ([_P(_VP), ctypes.c_int32], ctypes.c_int),
    "lar_depos_nonfinite": ([_P(lar_depos), _VP, _VP], ctypes.c_int),
    "lar_atomic_probe": ([_VP, ctypes.c_int64, ctypes.c_int64, _VP], ctypes.c_int),
    "lar_philox_probe": ([_VP, ctypes.c_int64, ctypes.c_int64, _VP], ctypes.c_int),
    "lar_row_copy_probe": ([_VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_int64, ctypes.c_int32,
                            ctypes.c_int32, _VP], ctypes.c_int),
    "lar_schedule_default": ([_P(lar_plane), _P(lar_schedule)], ctypes.c_int),
    "lar_schedule_get": ([_P(lar_plane), _P(lar_schedule)], ctypes.c_int),
    "lar_schedule_set": ([_P(lar_plane), _P(lar_schedule)], ctypes.c_int),
    "lar_schedule_candidates": ([_P(lar_plane), _P(lar_schedule), ctypes.c_int32, _P(ctypes.c_int32)],
                                ctypes.c_int),
    "lar_sample_counts": ([ctypes.c_int32, ctypes.c_int64, _VP, _VP, _VP, ctypes.c_uint32, ctypes.c_uint64,
                           _VP, _VP], ctypes.c_int),
    "lar_drift": ([_P(lar_drift_params), _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, _P(lar_plane_proj),
                   ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "lar_drift_backward_workspace": ([ctypes.c_int64, _P(_SZ)], ctypes.c_int),
    "lar_drift_backward": ([_P(lar_drift_params), _VP, _VP, ctypes.c_int64, _P(lar_plane_proj), ctypes.c_int32]
                           + [_VP] * 11 + [_VP, _SZ, _VP], ctypes.c_int),
    "lar_noise_workspace": ([_P(lar_plane), _P(_SZ)], ctypes.c_int),
    "lar_noise": ([_P(lar_plane), _VP, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _SZ, _VP],
                  ctypes.c_int),
    "lar_digitize": ([_VP, _VP, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _VP, _VP],
                     ctypes.c_int),
}

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2203_02479_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def lib():
    return _lib()


def _check(status, what):
    if status != LAR_OK:
        raise LarError(status, what)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_plane(p) -> lar_plane:
    """lar_plane from any object with the geometry attributes (e.g. inputs.Plane)."""
    return lar_plane(int(p.n_wires), int(p.n_imp), int(p.n_ticks), int(p.nt_fft), int(p.nw_fft),
                     float(p.pitch), float(p.x0), float(p.tick), float(p.t0))


class DeviceDepos:
    """Depositions resident on the GPU as five float32 tensors (SoA)."""

    def __init__(self, q, t, x, sigma_t, sigma_x):
        self.q, self.t, self.x, self.sigma_t, self.sigma_x = q, t, x, sigma_t, sigma_x
        n = q.numel()
        for a in (q, t, x, sigma_t, sigma_x):
            if a.dtype != torch.float32 or a.numel() != n or not a.is_cuda:
                raise TypeError("five float32 device tensors of equal length expected")

    @classmethod
    def from_host(cls, depos, device="cuda"):
        return cls(*(torch.as_tensor(a, dtype=torch.float32).to(device).contiguous() for a in depos.arrays()))

    def __len__(self):
        return self.q.numel()

    def struct(self) -> lar_depos:
        n = self.q.numel()
        if n == 0:
            return lar_depos(None, None, None, None, None, 0)
        return lar_depos(*(a.data_ptr() for a in (self.q, self.t, self.x, self.sigma_t, self.sigma_x)), n)


def _fluct(fluct):
    if fluct is None:
        return None
    if isinstance(fluct, lar_fluct):
        return ctypes.byref(fluct)
    mode, seed, event, plane = fluct
    return ctypes.byref(lar_fluct(int(mode), int(event), int(plane), 0, int(seed)))


def workspace(nbytes, device="cuda"):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- calls

def depos_nonfinite(depos: DeviceDepos, out=None, stream=None):
    """Number of depositions with a non-finite field (the ones the raster
    skips), counted on the GPU into out (a one-element int64 device tensor,
    allocated when None).  Returns out; out.item() synchronises."""
    if out is None:
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
    ds = depos.struct()
    _check(_lib().lar_depos_nonfinite(ctypes.byref(ds), _ptr(out), _stream(stream)), "lar_depos_nonfinite")
    return out


def atomic_probe(buf, n_segments, stream=None):
    """Peak-rate probe of the raster's global float atomics: adds 1 to
    n_segments scattered 64-float segments of buf (a float32 device tensor)."""
    if buf.dtype != torch.float32:
        raise TypeError("float32 buffer expected")
    _check(_lib().lar_atomic_probe(_ptr(buf), buf.numel(), int(n_segments), _stream(stream)), "lar_atomic_probe")


def philox_probe(out, n_blocks, stream=None):
    """Rate probe of the raster's per-bin draw: out (float64 device tensor,
    a multiple of 256 entries, one per thread) receives each thread's sum of
    the first uniforms of its Philox blocks, n_blocks blocks in all."""
    if out.dtype != torch.float64:
        raise TypeError("float64 output expected")
    _check(_lib().lar_philox_probe(_ptr(out), out.numel(), int(n_blocks), _stream(stream)), "lar_philox_probe")


def row_copy_probe(src, dst, n_out, blocks_per_cu=2, stream=None):
    """Memory-floor probe of the time R2C's access pattern: every row of src
    (float32 [rows][n_in]) read as float pairs, the first n_out complex
    values of every row of dst (float32 [rows][2 ld_out], complex values as
    float pairs, n_out <= ld_out) written."""
    if src.dtype != torch.float32 or dst.dtype != torch.float32 or src.dim() != 2 or dst.dim() != 2:
        raise TypeError("2-D float32 tensors expected")
    if src.shape[0] != dst.shape[0] or dst.shape[1] % 2:
        raise ValueError("row counts differ or odd output width")
    rows, n_in, ld_out = src.shape[0], src.shape[1], dst.shape[1] // 2
    _check(_lib().lar_row_copy_probe(_ptr(src), n_in, n_in, rows, _ptr(dst), ld_out, int(n_out),
                                     int(blocks_per_cu), _stream(stream)), "lar_row_copy_probe")


def raster_workspace(plane, n_depos, fluct) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_raster_workspace(ctypes.byref(make_plane(plane)), int(n_depos), _fluct(fluct),
                                       ctypes.byref(n)), "lar_raster_workspace")
    return n.value


def raster(plane, depos: DeviceDepos, nsigma, fluct, grid, ws=None, stream=None):
    pl = make_plane(plane)
    ds = depos.struct()
    wsp, wsn = (None, 0) if ws is None else (_ptr(ws), ws.numel())
    _check(_lib().lar_raster(ctypes.byref(pl), ctypes.byref(ds), float(nsigma), _fluct(fluct), _ptr(grid),
                             wsp, wsn, _stream(stream)), "lar_raster")


def fftconv_workspace(plane) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_fftconv_workspace(ctypes.byref(make_plane(plane)), ctypes.byref(n)),
           "lar_fftconv_workspace")
    return n.value


def fftconv(plane, grid, resp, wave, ws, stream=None):
    pl = make_plane(plane)
    _check(_lib().lar_fftconv(ctypes.byref(pl), _ptr(grid), _ptr(resp), _ptr(wave), _ptr(ws), ws.numel(),
                              _stream(stream)), "lar_fftconv")


def fftconv_noalloc(plane, grid, resp, wave, stream=None):
    """lar_fftconv without a workspace (the library's fixed device array)."""
    pl = make_plane(plane)
    _check(_lib().lar_fftconv_noalloc(ctypes.byref(pl), _ptr(grid), _ptr(resp), _ptr(wave), _stream(stream)),
           "lar_fftconv_noalloc")


def fftconv_noalloc_max_bytes() -> int:
    return int(_lib().lar_fftconv_noalloc_max_bytes())


def sim_plane_workspace(plane, n_depos=0, fluct=None) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_sim_plane_workspace(ctypes.byref(make_plane(plane)), int(n_depos), _fluct(fluct),
                                          ctypes.byref(n)), "lar_sim_plane_workspace")
    return n.value


def sim_plane(plane, depos: DeviceDepos, nsigma, fluct, resp, wave, ws, stream=None):
    pl = make_plane(plane)
    ds = depos.struct()
    _check(_lib().lar_sim_plane(ctypes.byref(pl), ctypes.byref(ds), float(nsigma), _fluct(fluct), _ptr(resp),
                                _ptr(wave), _ptr(ws), ws.numel(), _stream(stream)), "lar_sim_plane")


def fftconv_backward_workspace(plane) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_fftconv_backward_workspace(ctypes.byref(make_plane(plane)), ctypes.byref(n)),
           "lar_fftconv_backward_workspace")
    return n.value


def fftconv_backward(plane, grid, resp, wave_grad, grid_grad, resp_grad, ws, stream=None):
    pl = make_plane(plane)
    _check(_lib().lar_fftconv_backward(ctypes.byref(pl), _ptr(grid), _ptr(resp), _ptr(wave_grad),
                                       _ptr(grid_grad), _ptr(resp_grad), _ptr(ws), ws.numel(),
                                       _stream(stream)), "lar_fftconv_backward")


def fftconv_backward_spec_workspace(plane) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_fftconv_backward_spec_workspace(ctypes.byref(make_plane(plane)), ctypes.byref(n)),
           "lar_fftconv_backward_spec_workspace")
    return n.value


def spectrum_ld(plane) -> int:
    """Row pitch (complex elements) of the grid spectrum lar_fftconv leaves at
    the start of its workspace."""
    return (plane.nt_fft // 2 + 1 + 15) // 16 * 16


def fftconv_backward_spec(plane, grid_spec, resp, wave_grad, grid_grad, resp_grad, ws, accumulate=False,
                          stream=None):
    """grid_spec: a device buffer holding the grid spectrum (e.g. the fftconv
    workspace after lar_fftconv); only read."""
    pl = make_plane(plane)
    _check(_lib().lar_fftconv_backward_spec(ctypes.byref(pl), _ptr(grid_spec), _ptr(resp), _ptr(wave_grad),
                                            _ptr(grid_grad), _ptr(resp_grad), 1 if accumulate else 0, _ptr(ws),
                                            ws.numel(), _stream(stream)), "lar_fftconv_backward_spec")


def raster_backward(plane, depos: DeviceDepos, nsigma, grid_grad, dq, dt, dx, dsigma_t, dsigma_x,
                    stream=None):
    pl = make_plane(plane)
    ds = depos.struct()
    _check(_lib().lar_raster_backward(ctypes.byref(pl), ctypes.byref(ds), float(nsigma), _ptr(grid_grad),
                                      _ptr(dq), _ptr(dt), _ptr(dx), _ptr(dsigma_t), _ptr(dsigma_x),
                                      _stream(stream)), "lar_raster_backward")


def response_spectrum_workspace(plane, half_w, n_rt) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_response_spectrum_workspace(ctypes.byref(make_plane(plane)), int(half_w), int(n_rt),
                                                  ctypes.byref(n)), "lar_response_spectrum_workspace")
    return n.value


def response_spectrum(plane, r_time, half_w, n_rt, resp, ws, stream=None):
    pl = make_plane(plane)
    _check(_lib().lar_response_spectrum(ctypes.byref(pl), _ptr(r_time), int(half_w), int(n_rt), _ptr(resp),
                                        _ptr(ws), ws.numel(), _stream(stream)), "lar_response_spectrum")


def sample_counts(mode, q, p, ctr3, plane_id, seed, out, stream=None):
    n = q.numel()
    _check(_lib().lar_sample_counts(int(mode), n, _ptr(q), _ptr(p), _ptr(ctr3), int(plane_id), int(seed),
                                    _ptr(out), _stream(stream)), "lar_sample_counts")


def _drift_args(params, proj):
    v, dl, dt, tau = (float(a) for a in params)
    pr = (lar_plane_proj * max(len(proj), 1))(*[lar_plane_proj(*(float(c) for c in row)) for row in proj])
    return lar_drift_params(v, dl, dt, tau), pr, len(proj)


def drift(params, q0, t0, xd, y, z, proj, q, t, sigma_t, sigma_x, x, stream=None):
    """params = (speed, D_L, D_T, lifetime); proj = rows (cos, sin, offset)
    per plane; x: [n_planes][n] device tensor (or None with no planes)."""
    prm, pr, npl = _drift_args(params, proj)
    _check(_lib().lar_drift(ctypes.byref(prm), _ptr(q0), _ptr(t0), _ptr(xd), _ptr(y), _ptr(z), q0.numel(), pr,
                            npl, _ptr(q), _ptr(t), _ptr(sigma_t), _ptr(sigma_x), _ptr(x), _stream(stream)),
           "lar_drift")


def drift_backward_workspace(n) -> int:
    nb = ctypes.c_size_t(0)
    _check(_lib().lar_drift_backward_workspace(int(n), ctypes.byref(nb)), "lar_drift_backward_workspace")
    return nb.value


def drift_backward(params, q0, xd, proj, gq, gt, gsigma_t, gsigma_x, gx, dq0, dt0, dxd, dy, dz, dparams, ws,
                   stream=None):
    prm, pr, npl = _drift_args(params, proj)
    wsp, wsn = (None, 0) if ws is None else (_ptr(ws), ws.numel())
    _check(_lib().lar_drift_backward(ctypes.byref(prm), _ptr(q0), _ptr(xd), q0.numel(), pr, npl, _ptr(gq),
                                     _ptr(gt), _ptr(gsigma_t), _ptr(gsigma_x), _ptr(gx), _ptr(dq0), _ptr(dt0),
                                     _ptr(dxd), _ptr(dy), _ptr(dz), _ptr(dparams), wsp, wsn, _stream(stream)),
           "lar_drift_backward")


def noise_workspace(plane) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().lar_noise_workspace(ctypes.byref(make_plane(plane)), ctypes.byref(n)), "lar_noise_workspace")
    return n.value


def noise(plane, amp, seed, event, plane_id, out, ws, stream=None):
    pl = make_plane(plane)
    _check(_lib().lar_noise(ctypes.byref(pl), _ptr(amp), int(seed), int(event), int(plane_id), _ptr(out), _ptr(ws),
                            ws.numel(), _stream(stream)), "lar_noise")


def digitize(wave, noise_, gain, baseline, bits, adc, stream=None):
    """adc: uint16 codes (a torch.int16 / uint16 tensor of wave's size)."""
    _check(_lib().lar_digitize(_ptr(wave), _ptr(noise_), wave.numel(), float(gain), float(baseline), int(bits),
                               _ptr(adc), _stream(stream)), "lar_digitize")


# ---------------------------------------------------------------- conveniences

def spectrum_from_time(plane, r_time_np, device="cuda"):
    """Response spectrum [n_imp][Wf][F][2] float32 on the device from a
    time-domain response [n_imp][2H+1][L] (numpy)."""
    r = torch.as_tensor(r_time_np, dtype=torch.float32).to(device).contiguous()
    n_imp, nrw, L = r.shape
    H = (nrw - 1) // 2
    resp = torch.empty((plane.n_imp, plane.nw_fft, plane.nt_fft // 2 + 1, 2), dtype=torch.float32, device=device)
    ws = workspace(response_spectrum_workspace(plane, H, L), device)
    response_spectrum(plane, r, H, L, resp, ws)
    return resp


def set_stage_events(events):
    """Record the given torch.cuda.Event objects (5) after each kernel stage
    of lar_sim_plane / lar_fftconv on this thread; None to stop."""
    if events is None:
        _check(_lib().lar_set_stage_events(None, 0), "lar_set_stage_events")
        return
    arr = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
    _check(_lib().lar_set_stage_events(arr, len(events)), "lar_set_stage_events")


# ---------------------------------------------------------------- schedules

def schedule_default(plane) -> dict:
    out = lar_schedule()
    _check(_lib().lar_schedule_default(ctypes.byref(make_plane(plane)), ctypes.byref(out)),
           "lar_schedule_default")
    return out.as_dict()


def schedule_get(plane) -> dict:
    out = lar_schedule()
    _check(_lib().lar_schedule_get(ctypes.byref(make_plane(plane)), ctypes.byref(out)), "lar_schedule_get")
    return out.as_dict()


def schedule_set(plane, sched):
    """Register sched (a dict with the lar_schedule fields) for this plane
    shape; None restores the built-in schedule."""
    ptr = None
    if sched is not None:
        ptr = ctypes.byref(lar_schedule(*(int(sched.get(k, 0)) for k in lar_schedule.FIELDS)))
    _check(_lib().lar_schedule_set(ctypes.byref(make_plane(plane)), ptr), "lar_schedule_set")


def schedule_candidates(plane) -> list:
    P = make_plane(plane)
    n = ctypes.c_int32(0)
    _check(_lib().lar_schedule_candidates(ctypes.byref(P), None, 0, ctypes.byref(n)), "lar_schedule_candidates")
    arr = (lar_schedule * max(n.value, 1))()
    _check(_lib().lar_schedule_candidates(ctypes.byref(P), arr, n.value, ctypes.byref(n)),
           "lar_schedule_candidates")
    return [arr[i].as_dict() for i in range(n.value)]


# ---------------------------------------------------------------- batching

def make_items(items):
    """items: sequence of (plane_type, event, plane, depo_offset, n_depos, wave_offset)."""
    arr = (lar_batch_item * len(items))()
    for i, (pt, ev, pl, off, n, woff) in enumerate(items):
        arr[i] = lar_batch_item(int(pt), int(ev), int(pl), 0, int(off), int(n), int(woff))
    return arr


def batch_workspace(planes, items, fluct=None, max_wave=0) -> int:
    """Workspace for waves of at most max_wave items per plane type (0: all)."""
    pls = (lar_plane * len(planes))(*[make_plane(p) for p in planes])
    its = make_items(items)
    n = ctypes.c_size_t(0)
    _check(_lib().lar_batch_workspace_waves(pls, len(planes), its, len(its), _fluct(fluct), int(max_wave),
                                            ctypes.byref(n)), "lar_batch_workspace_waves")
    return n.value


class Batch:
    """A batch plan over fixed device buffers (depos concatenated, one
    response spectrum per plane type, one output buffer)."""

    def __init__(self, planes, resps, depos: DeviceDepos, nsigma, fluct, items, wave, ws, use_graph=True):
        self._keep = (resps, depos, wave, ws)
        pls = (lar_plane * len(planes))(*[make_plane(p) for p in planes])
        rp = (ctypes.c_void_p * len(resps))(*[r.data_ptr() for r in resps])
        its = make_items(items)
        ds = depos.struct()
        h = ctypes.c_void_p(0)
        _check(_lib().lar_batch_create(pls, len(planes), rp, ctypes.byref(ds), float(nsigma), _fluct(fluct), its,
                                       len(its), _ptr(wave), _ptr(ws), ws.numel(), 1 if use_graph else 0,
                                       ctypes.byref(h)), "lar_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(_lib().lar_batch_run(self._h, _stream(stream)), "lar_batch_run")

    def waves(self):
        """(number of waves, items in the largest wave)."""
        n, m = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib().lar_batch_waves(self._h, ctypes.byref(n), ctypes.byref(m)), "lar_batch_waves")
        return n.value, m.value

    def backward(self, wave_grad, resp_grads=None, depo_grads=None, stream=None):
        """resp_grads: one tensor per plane type (or None); depo_grads: five
        tensors in the depo layout (dq, dt, dx, dsigma_t, dsigma_x) or None."""
        rg = None
        if resp_grads is not None:
            rg = (ctypes.c_void_p * len(resp_grads))(*[None if r is None else r.data_ptr() for r in resp_grads])
        dg = [None] * 5 if depo_grads is None else [_ptr(d) for d in depo_grads]
        _check(_lib().lar_batch_backward(self._h, _ptr(wave_grad), rg, *dg, _stream(stream)), "lar_batch_backward")

    def close(self):
        if self._h:
            _lib().lar_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- streams

def sim_streams_workspace(planes, items, fluct, n_streams) -> int:
    pls = (lar_plane * len(planes))(*[make_plane(p) for p in planes])
    its = make_items(items)
    n = ctypes.c_size_t(0)
    _check(_lib().lar_sim_streams_workspace(pls, len(planes), its, len(its), _fluct(fluct), int(n_streams),
                                            ctypes.byref(n)), "lar_sim_streams_workspace")
    return n.value


def sim_streams(planes, resps, depos: DeviceDepos, nsigma, fluct, items, wave, streams, ws, stream=None):
    """Items as independent lar_sim_plane calls spread over `streams`
    (torch.cuda.Stream objects, default priority), joined back to `stream`."""
    pls = (lar_plane * len(planes))(*[make_plane(p) for p in planes])
    rp = (ctypes.c_void_p * len(resps))(*[r.data_ptr() for r in resps])
    its = make_items(items)
    ds = depos.struct()
    sp = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
    _check(_lib().lar_sim_streams(pls, len(planes), rp, ctypes.byref(ds), float(nsigma), _fluct(fluct), its, len(its),
                                  _ptr(wave), sp, len(streams), _ptr(ws), ws.numel(), _stream(stream)),
           "lar_sim_streams")
