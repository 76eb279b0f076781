// stages.hip -- the stages beside the raster and the convolution, for gfx950:
//
//  k_drift / k_drift_bwd  the drift of ionization groups to the anode
//               (paper Sec. 2.2: each group is diffused while it drifts,
//               into a 2D Gaussian over drift time and wire pitch): arrival
//               time, longitudinal and transverse widths from the diffusion
//               constants, charge attenuated by the electron lifetime, and
//               the pitch coordinate on every wire plane; and its adjoint,
//               with the parameter gradients reduced in a fixed order.
//  k_noise_spectrum  the noise term N(t,x) of Eq. (1): a random half
//               spectrum per wire (amplitude x complex standard normal),
//               inverse-transformed by the time-axis C2R kernel.
//  k_digitize   the ADC: waveform (plus noise) to integer codes.
//
// All three are elementwise and bound by HBM traffic (the noise spectrum's
// Philox and Box-Muller work is small next to the transform that follows).
// Arithmetic is FP64 without contraction where a CPU implementation of the
// same definition is meant to agree to the last float32 bit.
#include "lar_internal.hpp"

namespace lar {

// ---------------------------------------------------------------- drift

__global__ __launch_bounds__(256) void k_drift(DriftConst C, const float* __restrict__ q0,
                                               const float* __restrict__ t0, const float* __restrict__ xd,
                                               const float* __restrict__ y, const float* __restrict__ z,
                                               int64_t n, float* __restrict__ q, float* __restrict__ t,
                                               float* __restrict__ st, float* __restrict__ sx,
                                               float* __restrict__ x) {
#pragma clang fp contract(off)
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const double xdv = (double)xd[i];
        const double td = (xdv < 0.0 ? 0.0 : xdv) / C.v;   // a NaN distance stays NaN
        const double att = C.tau > 0.0 ? exp(-td / C.tau) : 1.0;
        q[i] = (float)((double)q0[i] * att);
        t[i] = (float)((double)t0[i] + td);
        st[i] = (float)(sqrt(2.0 * C.DL * td) / C.v);
        sx[i] = (float)sqrt(2.0 * C.DT * td);
        const double yv = (double)y[i], zv = (double)z[i];
        for (int p = 0; p < C.n_planes; ++p)
            x[(int64_t)p * n + i] = (float)(zv * C.proj[p][0] + yv * C.proj[p][1] + C.proj[p][2]);
    }
}

// Sum of a double over the workgroup (256 threads); thread 0 gets the total.
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// Adjoint of k_drift for L = sum(gq q + gt t + gst sigma_t + gsx sigma_x +
// sum_p gx_p x_p).  Where a width is zero its terms through the square root
// are zero (a point charge).  Parameter partials of each workgroup go to
// part[block][4] (v, D_L, D_T, tau); k_drift_reduce sums them in block order.
__global__ __launch_bounds__(256) void k_drift_bwd(
    DriftConst C, const float* __restrict__ q0, const float* __restrict__ xd, int64_t n,
    const float* __restrict__ gq, const float* __restrict__ gt, const float* __restrict__ gst,
    const float* __restrict__ gsx, const float* __restrict__ gx, float* __restrict__ dq0,
    float* __restrict__ dt0, float* __restrict__ dxd, float* __restrict__ dy, float* __restrict__ dz,
    double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    double pv = 0.0, pdl = 0.0, pdt = 0.0, ptau = 0.0;
    const double v = C.v, DL = C.DL, DT = C.DT, tau = C.tau;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const double xdv = (double)xd[i];
        const bool pos = xdv > 0.0;
        const double td = (pos ? xdv : 0.0) / v;
        const double att = tau > 0.0 ? exp(-td / tau) : 1.0;
        const double s = sqrt(2.0 * DL * td), sxv = sqrt(2.0 * DT * td);
        const double inv_s = s > 0.0 ? 1.0 / s : 0.0, inv_sx = sxv > 0.0 ? 1.0 / sxv : 0.0;
        const double q0v = (double)q0[i];
        const double g_q = (double)gq[i], g_t = (double)gt[i];
        const double g_st = (double)gst[i], g_sx = (double)gsx[i];
        const double dq_dtd = tau > 0.0 ? -q0v * att / tau : 0.0;
        const double g_td = g_q * dq_dtd + g_t + g_st * (DL * inv_s / v) + g_sx * (DT * inv_sx);
        if (dq0) dq0[i] = (float)(g_q * att);
        if (dt0) dt0[i] = (float)g_t;
        if (dxd) dxd[i] = (float)(pos ? g_td / v : 0.0);
        if (dy || dz) {
            double ay = 0.0, az = 0.0;
            for (int p = 0; p < C.n_planes; ++p) {
                const double g = (double)gx[(int64_t)p * n + i];
                ay += g * C.proj[p][1];
                az += g * C.proj[p][0];
            }
            if (dy) dy[i] = (float)ay;
            if (dz) dz[i] = (float)az;
        }
        pv += g_td * (-td / v) + g_st * (-s / (v * v));
        pdl += g_st * td * inv_s / v;
        pdt += g_sx * td * inv_sx;
        if (tau > 0.0) ptau += g_q * q0v * att * td / (tau * tau);
    }
    if (!part) return;
    pv = block_sum(pv, red);
    pdl = block_sum(pdl, red);
    pdt = block_sum(pdt, red);
    ptau = block_sum(ptau, red);
    if (threadIdx.x == 0) {
        double* o = part + 4 * (int64_t)blockIdx.x;
        o[0] = pv; o[1] = pdl; o[2] = pdt; o[3] = ptau;
    }
}

// Sums the nb partial rows in block order (one thread per parameter).
__global__ void k_drift_reduce(const double* __restrict__ part, int nb, float* __restrict__ dparams) {
    const int k = threadIdx.x;
    if (k >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[4 * b + k];
    dparams[k] = (float)s;
}

static int drift_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < kDriftMaxBlocks ? b : kDriftMaxBlocks);
}

hipError_t launch_drift(const DriftConst& C, const float* q0, const float* t0, const float* xd,
                        const float* y, const float* z, int64_t n, float* q, float* t, float* st,
                        float* sx, float* x, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_drift, dim3(drift_blocks(n)), dim3(256), 0, s, C, q0, t0, xd, y, z, n, q, t,
                       st, sx, x);
    return hipGetLastError();
}

hipError_t launch_drift_bwd(const DriftConst& C, const float* q0, const float* xd, int64_t n,
                            const float* gq, const float* gt, const float* gst, const float* gsx,
                            const float* gx, float* dq0, float* dt0, float* dxd, float* dy, float* dz,
                            float* dparams, double* part, hipStream_t s) {
    if (n <= 0) {   // no groups: zero parameter gradients
        if (dparams) hipLaunchKernelGGL(k_drift_reduce, dim3(1), dim3(64), 0, s, part, 0, dparams);
        return hipGetLastError();
    }
    const int nb = drift_blocks(n);
    hipLaunchKernelGGL(k_drift_bwd, dim3(nb), dim3(256), 0, s, C, q0, xd, n, gq, gt, gst, gsx, gx, dq0,
                       dt0, dxd, dy, dz, dparams ? part : nullptr);
    if (dparams) hipLaunchKernelGGL(k_drift_reduce, dim3(1), dim3(64), 0, s, part, nb, dparams);
    return hipGetLastError();
}

// ---------------------------------------------------------------- noise

// X[w][f] = amp[f] (g_re + i g_im) for wire w < n_wires and bin f < F, the
// normal pair from Box-Muller (cosine and sine branches) on the two
// uniforms of Philox block (w, event, f, plane*2^24 + 2^23): bit 23 of the
// last counter word marks the noise domain, which the raster's draw index
// never reaches.  The DC and Nyquist bins are real.
__global__ __launch_bounds__(256) void k_noise_spectrum(const float* __restrict__ amp, int F, int n_wires,
                                                        uint64_t seed, uint32_t event, uint32_t plane,
                                                        float2* __restrict__ X, int64_t ld) {
#pragma clang fp contract(off)
    const int64_t total = (int64_t)n_wires * F;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
        const int w = (int)(i / F), f = (int)(i - (int64_t)w * F);
        uint32_t c0 = (uint32_t)w, c1 = event, c2 = (uint32_t)f, c3 = (plane << 24) + 0x00800000u;
        philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u1 = u52(c0, c1), u2 = u52(c2, c3);
        const double r = sqrt(-2.0 * log(u1));
        const double a = 6.283185307179586 * u2;
        const double A = (double)amp[f];
        const bool real = f == 0 || f == F - 1;
        X[(int64_t)w * ld + f] = make_float2((float)(A * (r * cos(a))), real ? 0.f : (float)(A * (r * sin(a))));
    }
}

hipError_t launch_noise_spectrum(const float* amp, int F, int n_wires, uint64_t seed, uint32_t event,
                                 uint32_t plane, float2* X, int64_t ld, hipStream_t s) {
    const int64_t total = (int64_t)n_wires * F;
    if (total <= 0) return hipSuccess;
    const int64_t b = (total + 255) / 256, cap = 8 * (int64_t)device_cus();
    hipLaunchKernelGGL(k_noise_spectrum, dim3((unsigned)(b < cap ? b : cap)), dim3(256), 0, s, amp, F,
                       n_wires, seed, event, plane, X, ld);
    return hipGetLastError();
}

// ---------------------------------------------------------------- ADC

// code = clip(rint(gain * v + baseline), 0, maxcode), v = wave (+ noise),
// every step a float32 operation rounded on its own (no fused multiply-add),
// rint ties to even; a NaN voltage gives code 0.
__global__ __launch_bounds__(256) void k_digitize(const float* __restrict__ wave, const float* __restrict__ noise,
                                                  int64_t n, float gain, float baseline, float maxcode,
                                                  uint16_t* __restrict__ out) {
#pragma clang fp contract(off)
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        float v = wave[i];
        if (noise) v = v + noise[i];
        float y = gain * v;
        y = y + baseline;
        float c = rintf(y);
        c = c > 0.f ? c : 0.f;          // also maps NaN to 0
        c = c < maxcode ? c : maxcode;
        out[i] = (uint16_t)c;
    }
}

hipError_t launch_digitize(const float* wave, const float* noise, int64_t n, float gain, float baseline,
                           int bits, uint16_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t b = (n + 255) / 256, cap = 16 * (int64_t)device_cus();
    const float maxcode = (float)((1u << bits) - 1u);
    hipLaunchKernelGGL(k_digitize, dim3((unsigned)(b < cap ? b : cap)), dim3(256), 0, s, wave, noise, n, gain,
                       baseline, maxcode, out);
    return hipGetLastError();
}

}  // namespace lar
