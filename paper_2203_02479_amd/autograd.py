"""Differentiable plane simulation: a torch.autograd.Function over the C ABI.

Forward: mean raster (no fluctuation) + FFT convolution -> waveforms.
Backward: lar_fftconv_backward_spec (grid and response-spectrum gradients)
from the grid's time spectrum, which the forward convolution leaves at the
start of its workspace and which is kept instead of the grid (it is what the
response-spectrum gradient needs, and keeping it saves transforming the grid
again); then lar_raster_backward (depo gradients), which recomputes each
depo's patch instead of storing it.

Gradient convention for the response spectrum: resp is a float32 tensor
[n_imp][nw_fft][nt_fft/2+1][2] of (re, im) pairs and its gradient holds
(dL/dRe, dL/dIm) in the same layout.
"""
from __future__ import annotations

import torch

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
