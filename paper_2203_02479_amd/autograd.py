"""Differentiable plane simulation: a torch.autograd.Function over the C ABI.

Forward: mean raster (no fluctuation) + FFT convolution -> waveforms.
Backward: lar_fftconv_backward_spec (grid and response-spectrum gradients)
from the grid's time spectrum, which the forward convolution leaves at the
start of its workspace and which is kept instead of the grid (it is what the
response-spectrum gradient needs, and keeping it saves transforming the grid
again); then lar_raster_backward (depo gradients), which recomputes each
depo's patch instead of storing it.  The kept spectrum is only read, so the
graph may be walked backward more than once (retain_graph=True).

Gradient convention for the response spectrum: resp is a float32 tensor
[n_imp][nw_fft][nt_fft/2+1][2] of (re, im) pairs and its gradient holds
(dL/dRe, dL/dIm) in the same layout.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import lar


class SimPlaneFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, t, x, sigma_t, sigma_x, resp, plane, nsigma):
        D = lar.DeviceDepos(*(a.detach().contiguous() for a in (q, t, x, sigma_t, sigma_x)))
        grid = torch.zeros((plane.n_wires * plane.n_imp, plane.n_ticks), dtype=torch.float32, device=q.device)
        lar.raster(plane, D, nsigma, None, grid)
        wave = torch.empty((plane.n_wires, plane.n_ticks), dtype=torch.float32, device=q.device)
        ws = lar.workspace(lar.fftconv_workspace(plane), q.device)
        resp_c = resp.detach().contiguous()
        lar.fftconv(plane, grid, resp_c, wave, ws)
        del grid
        ctx.save_for_backward(D.q, D.t, D.x, D.sigma_t, D.sigma_x, resp_c, ws)   # ws: grid spectrum
        ctx.plane, ctx.nsigma = plane, nsigma
        return wave

    @staticmethod
    @once_differentiable
    def backward(ctx, gwave):
        q, t, x, st, sx, resp, spec = ctx.saved_tensors
        plane, nsigma = ctx.plane, ctx.nsigma
        need_depo = any(ctx.needs_input_grad[:5])
        need_resp = ctx.needs_input_grad[5]
        dev = gwave.device
        grid_grad = (torch.empty((plane.n_wires * plane.n_imp, plane.n_ticks), dtype=torch.float32, device=dev)
                     if need_depo else None)
        resp_grad = torch.empty_like(resp) if need_resp else None      # overwritten
        ws = lar.workspace(lar.fftconv_backward_spec_workspace(plane), dev)
        lar.fftconv_backward_spec(plane, spec, resp, gwave.contiguous(), grid_grad, resp_grad, ws)
        grads = [None] * 5
        if need_depo:
            grads = [torch.empty_like(q) for _ in range(5)]
            lar.raster_backward(plane, lar.DeviceDepos(q, t, x, st, sx), nsigma, grid_grad, *grads)
        return (*grads, resp_grad, None, None)


def sim_plane(q, t, x, sigma_t, sigma_x, resp, plane, nsigma=3.0):
    """Waveforms [n_wires][n_ticks] of one plane, differentiable with respect
    to the five depo arrays and the response spectrum."""
    return SimPlaneFunction.apply(q, t, x, sigma_t, sigma_x, resp, plane, nsigma)


class DriftFunction(torch.autograd.Function):
    """The drift stage (lar_drift) with its adjoint (lar_drift_backward):
    differentiable in the groups' inputs and in the parameters (speed, D_L,
    D_T, lifetime).  The parameters are read to the host (they are the call's
    scalar arguments)."""

    @staticmethod
    def forward(ctx, q0, t0, xd, y, z, params, proj):
        n = q0.numel()
        dev = q0.device
        arrs = [a.detach().contiguous() for a in (q0, t0, xd, y, z)]
        prm = [float(v) for v in params.detach().cpu().tolist()]
        outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4)]
        x = torch.empty((len(proj), n), dtype=torch.float32, device=dev)
        lar.drift(prm, *arrs, proj, *outs, x if len(proj) else None)
        ctx.save_for_backward(arrs[0], arrs[2])
        ctx.prm, ctx.proj, ctx.pdev = prm, proj, params.device
        return (*outs, x)

    @staticmethod
    @once_differentiable
    def backward(ctx, gq, gt, gst, gsx, gx):
        q0, xd = ctx.saved_tensors
        n, dev = q0.numel(), q0.device
        z = lambda g, shape: (torch.zeros(shape, dtype=torch.float32, device=dev) if g is None
                              else g.contiguous())
        gq, gt, gst, gsx = (z(g, (n,)) for g in (gq, gt, gst, gsx))
        gx = z(gx, (len(ctx.proj), n))
        need = ctx.needs_input_grad
        outs = [torch.empty(n, dtype=torch.float32, device=dev) if need[i] else None for i in range(5)]
        dparams = torch.empty(4, dtype=torch.float32, device=dev) if need[5] else None
        ws = lar.workspace(lar.drift_backward_workspace(n), dev) if dparams is not None else None
        lar.drift_backward(ctx.prm, q0, xd, ctx.proj, gq, gt, gst, gsx, gx if len(ctx.proj) else None, *outs,
                           dparams, ws)
        if dparams is not None:
            dparams = dparams.to(ctx.pdev)
        return (*outs, dparams, None)


def drift(q0, t0, xd, y, z, params, proj):
    """Drifted groups (q, t, sigma_t, sigma_x, x[n_planes]) from undrifted
    ones; params = tensor (speed, D_L, D_T, lifetime), proj = rows (cos,
    sin, offset) per plane."""
    return DriftFunction.apply(q0, t0, xd, y, z, params, tuple(tuple(float(c) for c in r) for r in proj))
