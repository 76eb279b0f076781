"""FP64 CPU oracle for the LArTPC signal-simulation hot path.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product (the GPU library and
its Python binding) never imports, links or runs it, and the two share no
code.

Contents (paper arXiv:2203.02479):

* ``raster_mean`` / ``raster_fluct`` / ``raster_adjoint`` -- the "Raster" and
  "Scatter-add" tasks (Sec. 2.2) in plain C (``lar_oracle.c``), FP64.
* ``sample_counts`` / ``philox`` / ``stream_uniforms`` -- the per-bin
  fluctuation (Sec. 3.1: the reference code samples a binomial).
* ``response_spectrum`` / ``conv_fft`` -- the frequency-domain convolution of
  Sec. 2.2 Eq. (2): FT of the charge grid, product with the response
  spectrum, inverse FT, with scipy's FFT (pocketfft) as the transform step.
* ``conv_direct`` -- Eq. (1) first term as a brute-force sum (tiny sizes).
* ``conv_adjoint`` -- gradients of <M, G> with respect to the grid and the
  complex response spectrum.
* ``sample_counts`` mode 3 -- the normal approximation of the binomial that
  the paper's GPU port uses (Sec. 3.1).
* ``stages.drift`` / ``drift_adjoint`` -- the drift stage upstream of the
  raster (Sec. 2.2); ``stages.noise`` / ``digitize`` -- the noise term of
  Eq. (1) and the ADC downstream of the convolution.

Conventions fixed where the paper is silent: the time axis is circular over
the FFT length Tf (ticks >= n_ticks hold zero charge), the wire axis circular
over Wf (linear when Wf >= n_wires + 2H); forward transforms are
unnormalised, the inverse carries 1/(Wf*Tf); the real inverse transform in
time takes the real part of the DC and Nyquist columns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.fft as sfft

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lar_oracle.c")
_SO = os.path.join(_HERE, "liblar_oracle.so")
_lib = None
_THREADS = 1          # threads of the C depo loops and of the FFT steps

_c = ctypes
_pf = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_pd = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_pu = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the C part of the oracle (gcc, -O2, no contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        geo = [_c.c_int, _c.c_int, _c.c_int, _c.c_double, _c.c_double, _c.c_double,
               _c.c_double, _c.c_double, _c.c_int64, _pf, _pf, _pf, _pf, _pf]
        L.lo_phi_diff.argtypes = [_c.c_double, _c.c_double]
        L.lo_phi_diff.restype = _c.c_double
        L.lo_axis.argtypes = [_c.c_double, _c.c_double, _c.c_double, _c.c_double, _c.c_double,
                              _c.c_int, _c.POINTER(_c.c_int), _pd, _pd, _pd]
        L.lo_axis.restype = _c.c_int
        L.lo_raster_mean.argtypes = geo + [_pd]
        L.lo_raster_fluct.argtypes = geo + [_c.c_int, _c.c_uint64, _c.c_uint32, _c.c_uint32, _pd]
        L.lo_raster_adjoint.argtypes = geo + [_pd, _pd, _pd, _pd, _pd, _pd]
        L.lo_philox4x32_10.argtypes = [_pu, _pu, _pu]
        L.lo_philox4x32_10.restype = None
        L.lo_u53.argtypes = [_c.c_uint32, _c.c_uint32]
        L.lo_u53.restype = _c.c_double
        L.lo_sample_counts.argtypes = [_c.c_int, _c.c_int64, _pf, _pd, _pu, _c.c_uint32,
                                       _c.c_uint64, _pd]
        L.lo_sample_counts.restype = None
        L.lo_stream_uniforms.argtypes = [_c.c_uint64, _c.c_uint32, _c.c_uint32, _c.c_uint32,
                                         _c.c_uint32, _c.c_int, _pd]
        L.lo_stream_uniforms.restype = None
        L.lo_conv_direct.argtypes = [_c.c_int] * 7 + [_pd, _pd, _pd]
        L.lo_conv_direct.restype = None
        L.lo_box_muller.argtypes = [_c.c_double, _c.c_double, _c.POINTER(_c.c_double),
                                    _c.POINTER(_c.c_double)]
        L.lo_box_muller.restype = None
        L.lo_set_threads.argtypes = [_c.c_int]
        L.lo_set_threads.restype = _c.c_int
        L.lo_set_threads(_THREADS)
        L.lo_fc.argtypes = [_c.c_double]
        L.lo_fc.restype = _c.c_double
        L.lo_btrd_log_accept.argtypes = [_c.c_double] * 4
        L.lo_btrd_log_accept.restype = _c.c_int
        L.lo_ptrs_log_accept.argtypes = [_c.c_double] * 4
        L.lo_ptrs_log_accept.restype = _c.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads for the oracle's depo loops (OpenMP) and FFT steps (scipy's
    pocketfft workers); 1 by default.  Only the order of FP64 sums changes."""
    global _THREADS
    _THREADS = max(1, int(n))
    lib().lo_set_threads(_THREADS)
    return _THREADS


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _geo(plane, depos, nsigma):
    q, t, x, st, sx = (_f32(a) for a in depos.arrays())
    return (int(plane.n_wires), int(plane.n_imp), int(plane.n_ticks), float(np.float32(plane.pitch)),
            float(np.float32(plane.x0)), float(np.float32(plane.tick)), float(np.float32(plane.t0)),
            float(np.float32(nsigma)), int(len(q)), q, t, x, st, sx)


# ------------------------------------------------------------------ raster

def phi_diff(za: float, zb: float) -> float:
    """Phi(zb) - Phi(za) (standard normal CDF), tail-safe."""
    return lib().lo_phi_diff(float(za), float(zb))


def axis(mu, sigma, nsig, origin, width, nbins):
    """One axis of a deposition: (lo, w, dw/dmu, dw/dsigma) over the window."""
    w = np.zeros(max(nbins, 1)); dmu = np.zeros_like(w); ds = np.zeros_like(w)
    lo = _c.c_int(0)
    n = lib().lo_axis(float(mu), float(sigma), float(nsig), float(origin), float(width),
                      int(nbins), _c.byref(lo), w, dmu, ds)
    return lo.value, w[:n].copy(), dmu[:n].copy(), ds[:n].copy()


def raster_mean(plane, depos, nsigma=3.0, grid=None):
    """Mean charge grid S [n_wires*n_imp][n_ticks] (float64), accumulated."""
    if grid is None:
        grid = np.zeros((plane.n_wires * plane.n_imp, plane.n_ticks))
    if lib().lo_raster_mean(*_geo(plane, depos, nsigma), grid) != 0:
        raise MemoryError("oracle raster")
    return grid


def raster_fluct(plane, depos, nsigma=3.0, mode=1, seed=0, event=0, plane_id=0, grid=None):
    """Fluctuated grid: sign(q) * Binomial(rint|q|, p) (mode 1) or
    sign(q) * Poisson(|q| p) (mode 2) per bin, accumulated."""
    if grid is None:
        grid = np.zeros((plane.n_wires * plane.n_imp, plane.n_ticks))
    if lib().lo_raster_fluct(*_geo(plane, depos, nsigma), int(mode), int(seed), int(event),
                             int(plane_id), grid) != 0:
        raise MemoryError("oracle raster")
    return grid


def raster_adjoint(plane, depos, nsigma, G):
    """(dq, dt, dx, dsigma_t, dsigma_x) of sum(G * S) for the mean grid."""
    n = len(depos)
    outs = [np.zeros(n) for _ in range(5)]
    G = np.ascontiguousarray(G, dtype=np.float64)
    dq, dt, dx, dst, dsx = outs
    if lib().lo_raster_adjoint(*_geo(plane, depos, nsigma), G, dq, dt, dx, dst, dsx) != 0:
        raise MemoryError("oracle raster")
    return dq, dt, dx, dst, dsx


# ------------------------------------------------------------------ random numbers

def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter and 2-word key."""
    out = np.zeros(4, np.uint32)
    lib().lo_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def u53(a, b):
    return lib().lo_u53(int(a), int(b))


def stream_uniforms(seed, depo, event, bin_, plane, count):
    out = np.zeros(count)
    lib().lo_stream_uniforms(int(seed), int(depo), int(event), int(bin_), int(plane), int(count), out)
    return out


def stirling_tail(k):
    """The samplers' fc(k) = log k! - [(k+1/2) log(k+1) - (k+1) + log(2 pi)/2]."""
    return lib().lo_fc(float(k))


def btrd_log_accept(n, p, k, v):
    """BTRD's decision for a try at k far from the mode (|k - m| > 15) with
    rescaled uniform v: True to accept (log v <= log f(k)/f(m))."""
    return bool(lib().lo_btrd_log_accept(float(n), float(p), float(k), float(v)))


def ptrs_log_accept(lam, us, v, k):
    """PTRS's final decision for candidate k with us = 1/2 - |u| and uniform v."""
    return bool(lib().lo_ptrs_log_accept(float(lam), float(us), float(v), float(k)))


def box_muller(u1, u2):
    """(sqrt(-2 log u1) cos(2 pi u2), sqrt(-2 log u1) sin(2 pi u2))."""
    c, s = _c.c_double(0.0), _c.c_double(0.0)
    lib().lo_box_muller(float(u1), float(u2), _c.byref(c), _c.byref(s))
    return c.value, s.value


def sample_counts(mode, q, p, ctr3, plane_id, seed):
    """Signed per-bin counts for injected (q, p, counter) triples: mode 1
    binomial, 2 Poisson, 3 normal approximation of the binomial.
    ctr3 is uint32 [n][3] = (depo, event, bin)."""
    q = _f32(q)
    p = np.ascontiguousarray(p, dtype=np.float64)
    ctr3 = np.ascontiguousarray(ctr3, dtype=np.uint32)
    out = np.zeros(len(q))
    lib().lo_sample_counts(int(mode), len(q), q, p, ctr3, int(plane_id), int(seed), out)
    return out


# ------------------------------------------------------------------ convolution

def resp_complex(resp):
    """Interleaved float32 (re, im) [..., 2] -> complex128."""
    r = np.asarray(resp)
    if np.iscomplexobj(r):
        return r.astype(np.complex128)
    r = r.astype(np.float64)
    return r[..., 0] + 1j * r[..., 1]


def response_spectrum(plane, r_time):
    """R_k = 2D DFT over (Wf, Tf) of r[k][dw + H][tau] placed at
    (dw mod Wf, tau): complex128 [n_imp][Wf][Tf/2+1]."""
    r = np.asarray(r_time, dtype=np.float64)
    n_imp, nw, L = r.shape
    H = (nw - 1) // 2
    Wf, Tf = plane.nw_fft, plane.nt_fft
    full = np.zeros((n_imp, Wf, Tf))
    for i in range(nw):
        full[:, (i - H) % Wf, :L] += r[:, i, :]
    return np.fft.fft(np.fft.rfft(full, axis=2), axis=1)


def _rfft2(plane, A):
    """rfft over time (length Tf) then FFT over wire (length Wf), zero padded."""
    w = _THREADS
    return sfft.fft(sfft.rfft(A, n=plane.nt_fft, axis=-1, workers=w), n=plane.nw_fft, axis=-2, workers=w)


def _irfft2_crop(plane, X):
    """Inverse FFT over wire, keep the first n_wires rows, real inverse over
    time with the DC and Nyquist columns taken as real, crop to n_ticks."""
    w = _THREADS
    Y = sfft.ifft(X, axis=-2, workers=w)[..., :plane.n_wires, :].copy()
    Y[..., 0] = Y[..., 0].real
    Y[..., -1] = Y[..., -1].real
    return sfft.irfft(Y, n=plane.nt_fft, axis=-1, workers=w)[..., :plane.n_ticks]


def sub_grids(plane, S):
    """S[w*n_imp + k][t] -> S_k[k][w][t]."""
    S = np.asarray(S, dtype=np.float64)
    return S.reshape(plane.n_wires, plane.n_imp, plane.n_ticks).transpose(1, 0, 2)


def conv_fft(plane, S, resp):
    """Waveforms M [n_wires][n_ticks] = crop irfft2( sum_k R_k * rfft2(S_k) )."""
    R = resp_complex(resp)
    acc = np.zeros((plane.nw_fft, plane.nt_fft // 2 + 1), np.complex128)
    Sk = sub_grids(plane, S)
    for k in range(plane.n_imp):
        acc += R[k] * _rfft2(plane, Sk[k])
    return _irfft2_crop(plane, acc)


def conv_adjoint(plane, S, resp, G):
    """Gradients of L = <M, G> (real inner product):
    grid gradient G_S [n_wires*n_imp][n_ticks] and response-spectrum gradient
    dR [n_imp][Wf][F] (complex, d/dRe + i d/dIm)."""
    R = resp_complex(resp)
    Gh = _rfft2(plane, np.asarray(G, np.float64))
    F = plane.nt_fft // 2 + 1
    cf = np.full(F, 2.0)
    cf[0] = 1.0
    cf[-1] = 1.0
    scale = cf / (plane.nw_fft * plane.nt_fft)
    Sk = sub_grids(plane, S)
    GS = np.zeros((plane.n_wires, plane.n_imp, plane.n_ticks))
    dR = np.zeros_like(R)
    for k in range(plane.n_imp):
        GS[:, k, :] = _irfft2_crop(plane, np.conj(R[k]) * Gh)
        dR[k] = scale[None, :] * Gh * np.conj(_rfft2(plane, Sk[k]))
    return GS.reshape(plane.n_wires * plane.n_imp, plane.n_ticks), dR


def conv_direct(plane, r_time, S):
    """Brute-force circular convolution (tiny sizes only)."""
    r = np.ascontiguousarray(r_time, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    n_imp, nw, L = r.shape
    M = np.zeros((plane.n_wires, plane.n_ticks))
    lib().lo_conv_direct(plane.n_wires, plane.n_imp, plane.n_ticks, plane.nw_fft, plane.nt_fft,
                         (nw - 1) // 2, L, r, S, M)
    return M


def sim_plane_mean(plane, depos, resp, nsigma=3.0):
    """Mean-path waveforms of one plane: conv_fft(raster_mean(...))."""
    return conv_fft(plane, raster_mean(plane, depos, nsigma), resp)


from .stages import (digitize, drift, drift_adjoint, noise, noise_digitize,  # noqa: E402
                     noise_normals, noise_spectrum)
