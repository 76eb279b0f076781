"""FP64 oracle of the stages beside the raster and the convolution: the drift
stage upstream of the path, and the noise term and digitisation downstream.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

* ``drift`` / ``drift_adjoint`` -- the drift of ionization groups to the
  anode (paper Sec. 2.2: each group is diffused while it drifts, into a 2D
  distribution over drift time and wire pitch).  Per group: arrival time
  t = t0 + td with td = max(xd, 0)/v, longitudinal width
  sigma_L = sqrt(2 D_L td)/v (time units), transverse width
  sigma_T = sqrt(2 D_T td), charge q = q0 exp(-td/tau) (electron lifetime
  tau; tau <= 0 means no attenuation), and for each plane the pitch
  coordinate x = z cos(theta) + y sin(theta) + offset.
* ``noise`` -- the noise term N(t,x) of Eq. (1): per wire, a random
  spectrum A(f) (g_re + i g_im) with independent standard normals per
  (wire, frequency), inverse real FFT over Tf (1/Tf normalisation, the
  imaginary parts of the DC and Nyquist bins dropped), cropped to n_ticks.
* ``digitize`` -- the ADC: code = clip(rint(gain*v + baseline), 0,
  2^bits - 1) with the products and sums in float32 (the precision the
  codes are decided in on the GPU) and rint rounding ties to even.
"""
from __future__ import annotations

import numpy as np

from . import lib, _pd
import ctypes as _c


# ------------------------------------------------------------------ drift

def _f32_exact(a):
    return np.asarray(a, np.float32).astype(np.float64)


def drift(params, q0, t0, xd, y, z, proj):
    """Drifted groups: (q, t, sigma_t, sigma_x, x[n_planes][n]) in float64,
    from the float32 values of every input (what the GPU receives).

    params = (v [mm/us], D_L [mm^2/us], D_T [mm^2/us], lifetime [us]);
    proj = [n_planes][3] rows (cos theta, sin theta, offset)."""
    return drift_f64(_f32_exact(params), *(_f32_exact(a) for a in (q0, t0, xd, y, z)),
                     _f32_exact(proj).reshape(-1, 3))


def drift_f64(params, q0, t0, xd, y, z, proj):
    """drift() on float64 inputs as given (for finite differences)."""
    v, DL, DT, tau = (float(p) for p in params)
    proj = np.asarray(proj, np.float64).reshape(-1, 3)
    td = np.maximum(xd, 0.0) / v
    att = np.exp(-td / tau) if tau > 0 else np.ones_like(td)
    q = q0 * att
    t = t0 + td
    sigma_t = np.sqrt(2.0 * DL * td) / v
    sigma_x = np.sqrt(2.0 * DT * td)
    x = np.stack([z * c + y * s + o for (c, s, o) in proj])
    return q, t, sigma_t, sigma_x, x


def drift_adjoint(params, q0, t0, xd, y, z, proj, gq, gt, gst, gsx, gx):
    """Gradients of L = sum(gq q + gt t + gst sigma_t + gsx sigma_x + sum_p gx_p x_p)
    with respect to the per-group inputs and the four parameters.

    Returns (dq0, dt0, dxd, dy, dz, dparams[4]).  Where a width is zero (no
    drift, or zero diffusion) its derivative terms through the square root
    are taken as zero, as for a point charge."""
    return drift_adjoint_f64(_f32_exact(params), *(_f32_exact(a) for a in (q0, t0, xd, y, z)),
                             _f32_exact(proj).reshape(-1, 3), gq, gt, gst, gsx, gx)


def drift_adjoint_f64(params, q0, t0, xd, y, z, proj, gq, gt, gst, gsx, gx):
    """drift_adjoint() on float64 inputs as given."""
    v, DL, DT, tau = (float(p) for p in params)
    gq, gt, gst, gsx = (np.asarray(a, np.float64) for a in (gq, gt, gst, gsx))
    proj = np.asarray(proj, np.float64).reshape(-1, 3)
    gx = np.asarray(gx, np.float64).reshape(len(proj), -1)
    pos = xd > 0.0
    td = np.where(pos, xd, 0.0) / v
    att = np.exp(-td / tau) if tau > 0 else np.ones_like(td)
    s = np.sqrt(2.0 * DL * td)                    # sigma_t * v
    sx = np.sqrt(2.0 * DT * td)
    inv_s = np.divide(1.0, s, out=np.zeros_like(s), where=s > 0)
    inv_sx = np.divide(1.0, sx, out=np.zeros_like(sx), where=sx > 0)
    dq_dtd = -q0 * att / tau if tau > 0 else np.zeros_like(td)
    dsl_dtd = DL * inv_s / v
    dsx_dtd = DT * inv_sx
    g_td = gq * dq_dtd + gt + gst * dsl_dtd + gsx * dsx_dtd
    dq0 = gq * att
    dt0 = gt.copy()
    dxd = np.where(pos, g_td / v, 0.0)
    dy = sum(gx[p] * proj[p, 1] for p in range(len(proj)))
    dz = sum(gx[p] * proj[p, 0] for p in range(len(proj)))
    d_v = np.sum(g_td * (-td / v) + gst * (-s / (v * v)))
    d_DL = np.sum(gst * td * inv_s / v)
    d_DT = np.sum(gsx * td * inv_sx)
    d_tau = np.sum(gq * q0 * att * td / (tau * tau)) if tau > 0 else 0.0
    return dq0, dt0, dxd, dy, dz, np.array([d_v, d_DL, d_DT, d_tau])


# ------------------------------------------------------------------ noise

def noise_normals(seed, event, plane_id, n_wires, nf):
    """Standard normal pairs (re, im) [n_wires][nf] of the noise spectrum."""
    L = lib()
    if not getattr(L, "_noise_bound", False):
        L.lo_noise_normals.argtypes = [_c.c_uint64, _c.c_uint32, _c.c_uint32, _c.c_int, _c.c_int, _pd, _pd]
        L.lo_noise_normals.restype = None
        L._noise_bound = True
    re = np.zeros((n_wires, nf))
    im = np.zeros((n_wires, nf))
    L.lo_noise_normals(int(seed), int(event), int(plane_id), int(n_wires), int(nf), re, im)
    return re, im


def noise_spectrum(plane, amp, seed, event, plane_id):
    """The random half spectrum X[w][f] = amp[f] (g_re + i g_im), with the
    DC and Nyquist bins real."""
    F = plane.nt_fft // 2 + 1
    amp = np.asarray(amp, np.float32).astype(np.float64)
    re, im = noise_normals(seed, event, plane_id, plane.n_wires, F)
    X = amp[None, :] * (re + 1j * im)
    X[:, 0] = amp[0] * re[:, 0]
    X[:, F - 1] = amp[F - 1] * re[:, F - 1]
    return X


def noise(plane, amp, seed, event, plane_id):
    """Noise waveforms [n_wires][n_ticks]: inverse real FFT over Tf of the
    random spectrum (1/Tf), cropped."""
    X = noise_spectrum(plane, amp, seed, event, plane_id)
    return np.fft.irfft(X, n=plane.nt_fft, axis=1)[:, :plane.n_ticks]


def digitize(v32, gain, baseline, bits):
    """ADC codes (uint16) of float32 voltages: rint(gain*v + baseline) in
    float32 operations (product rounded, then sum rounded), clipped to
    [0, 2^bits - 1]."""
    v32 = np.asarray(v32, np.float32)
    g, b = np.float32(gain), np.float32(baseline)
    y = (g * v32).astype(np.float32)
    y = (y + b).astype(np.float32)
    c = np.rint(y.astype(np.float64))
    c = np.clip(c, 0.0, float(2 ** int(bits) - 1))
    return c.astype(np.uint16)


def noise_digitize(plane, wave32, amp, seed, event, plane_id, gain, baseline, bits):
    """Codes of waveforms plus noise: digitize(float32(wave + float32(noise)))."""
    n32 = noise(plane, amp, seed, event, plane_id).astype(np.float32)
    v = (np.asarray(wave32, np.float32) + n32).astype(np.float32)
    return digitize(v, gain, baseline, bits)
