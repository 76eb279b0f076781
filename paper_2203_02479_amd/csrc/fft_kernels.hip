// fft_kernels.hip -- frequency-domain convolution of the charge grid with the
// detector response (paper Sec. 2.2 Eq. (2)) for gfx950.
//
//  k_r2c_rows   real FFT along ticks of every grid row (length Tf, as a
//               Tf/2-point complex FFT of even/odd pairs plus the split step)
//  k_wire_fused per tile of time-frequency columns: for each impact offset k,
//               gather the rows w*n_imp + k, FFT over wires (Wf), multiply by
//               the response spectrum of offset k and accumulate; then one
//               inverse FFT over wires.  The impact-offset reduction never
//               leaves the chip.
//  k_c2r_rows   inverse real FFT along ticks, scaled by 1/(Wf Tf), cropped.
//
// All three are bound by HBM traffic: every transform lives in LDS and each
// grid element is read and written once per pass.
#include "lar_internal.hpp"

namespace lar {

bool make_plan(int n, FftPlan* plan) {
    if (n < 1) return false;
    int m = n, np = 0;
    while (m % 4 == 0 && np < kMaxPasses) { plan->radix[np++] = 4; m /= 4; }
    while (m % 3 == 0 && np < kMaxPasses) { plan->radix[np++] = 3; m /= 3; }
    while (m % 2 == 0 && np < kMaxPasses) { plan->radix[np++] = 2; m /= 2; }
    if (m != 1) return false;
    plan->n = n;
    plan->npass = np;
    return true;
}

int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

static constexpr int kRowThreads = 256;

// Half-angle table h[k] = exp(-pi i k / Nh) = exp(-2 pi i k / Tf), k < Nh,
// computed in double and rounded once.
__device__ __forceinline__ void fill_half_table(float2* h, int Nh, int tid, int T) {
    for (int i = tid; i < Nh; i += T) {
        double s, c;
        sincospi(-(double)i / (double)Nh, &s, &c);
        h[i] = make_float2((float)c, (float)s);
    }
}

template <int VPT>
__global__ __launch_bounds__(kRowThreads) void k_r2c_rows(const float* __restrict__ in,
                                                          int64_t ld_in, int n_in, int nrows,
                                                          FftPlan plan, float2* __restrict__ out,
                                                          int64_t ld_out, int pairs_ok) {
    extern __shared__ float2 lds[];
    const int Nh = plan.n, tid = threadIdx.x, T = blockDim.x;
    float2* A = lds;
    float2* h = lds + Nh;
    fill_half_table(h, Nh, tid, T);
    const TwHalf tw{h, Nh};
    for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
        const float* x = in + (int64_t)row * ld_in;
        __syncthreads();
        if (pairs_ok) {
            const float2* x2 = reinterpret_cast<const float2*>(x);
            const int full = n_in >> 1;
            for (int n = tid; n < Nh; n += T) {
                float2 v = make_float2(0.f, 0.f);
                if (n < full) v = x2[n];
                else if (2 * n < n_in) v.x = x[2 * n];
                A[n] = v;
            }
        } else {
            for (int n = tid; n < Nh; n += T) {
                int i0 = 2 * n;
                A[n] = make_float2(i0 < n_in ? x[i0] : 0.f, i0 + 1 < n_in ? x[i0 + 1] : 0.f);
            }
        }
        __syncthreads();
        fft_lds<VPT, 1>(A, plan, tid, T, tw, false);
        // split step: X[k] = (Z[k] + Z*[Nh-k])/2 - i W^k (Z[k] - Z*[Nh-k])/2
        float2* y = out + (int64_t)row * ld_out;
        for (int k = tid; k <= Nh / 2; k += T) {
            float2 zk = A[k], zm = A[k == 0 ? 0 : Nh - k];
            float2 w = h[k];
            float2 e1 = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            float2 d1 = make_float2(zk.x - zm.x, zk.y + zm.y);
            float2 wd1 = cmul(w, d1);
            float2 xk = make_float2(e1.x + 0.5f * wd1.y, e1.y - 0.5f * wd1.x);
            float2 e2 = make_float2(0.5f * (zm.x + zk.x), 0.5f * (zm.y - zk.y));
            float2 d2 = make_float2(zm.x - zk.x, zm.y + zk.y);
            float2 wd2 = cmul(make_float2(-w.x, w.y), d2);    // W^(Nh-k) = -conj(W^k)
            float2 xm = make_float2(e2.x + 0.5f * wd2.y, e2.y - 0.5f * wd2.x);
            y[k] = xk;
            y[Nh - k] = xm;
        }
    }
}

template <int VPT>
__global__ __launch_bounds__(kRowThreads) void k_c2r_rows(const float2* __restrict__ in,
                                                          int64_t ld_in, int nrows, FftPlan plan,
                                                          float* __restrict__ out, int64_t ld_out,
                                                          int n_out, float scale, int pairs_ok) {
    extern __shared__ float2 lds[];
    const int Nh = plan.n, tid = threadIdx.x, T = blockDim.x;
    float2* A = lds;
    float2* h = lds + Nh;
    fill_half_table(h, Nh, tid, T);
    const TwHalf tw{h, Nh};
    for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
        const float2* X = in + (int64_t)row * ld_in;
        __syncthreads();
        // pre-step: Z[k] = (X[k] + X*[Nh-k]) + i (X[k] - X*[Nh-k]) exp(+2 pi i k/Tf),
        // the imaginary parts of the DC and Nyquist bins are dropped
        for (int k = tid; k <= Nh / 2; k += T) {
            float2 xk = X[k], xm = X[Nh - k];
            if (k == 0) { xk.y = 0.f; xm.y = 0.f; }
            float2 w = h[k];
            float2 a1 = make_float2(xk.x + xm.x, xk.y - xm.y);
            float2 b1 = cmulc(make_float2(xk.x - xm.x, xk.y + xm.y), w);   // * exp(+2 pi i k/Tf)
            float2 a2 = make_float2(xm.x + xk.x, xm.y - xk.y);
            float2 b2 = cmul(make_float2(xm.x - xk.x, xm.y + xk.y), make_float2(-w.x, -w.y));
            A[k] = make_float2(a1.x - b1.y, a1.y + b1.x);
            if (k > 0) A[Nh - k] = make_float2(a2.x - b2.y, a2.y + b2.x);
        }
        __syncthreads();
        fft_lds<VPT, 1>(A, plan, tid, T, tw, true);
        float* y = out + (int64_t)row * ld_out;
        if (pairs_ok) {
            float2* y2 = reinterpret_cast<float2*>(y);
            const int full = n_out >> 1;
            for (int n = tid; n < Nh; n += T) {
                float2 z = A[n];
                if (n < full) y2[n] = make_float2(z.x * scale, z.y * scale);
                else if (2 * n < n_out) y[2 * n] = z.x * scale;
            }
        } else {
            for (int n = tid; n < Nh; n += T) {
                float2 z = A[n];
                if (2 * n < n_out) y[2 * n] = z.x * scale;
                if (2 * n + 1 < n_out) y[2 * n + 1] = z.y * scale;
            }
        }
    }
}

template <class K>
static void set_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static int row_grid(int nrows) {
    int g = 4 * device_cus();
    return nrows < g ? nrows : g;
}

hipError_t launch_r2c_rows(const float* in, int64_t ld_in, int n_in, int nrows, int nt_fft,
                           float2* out, int64_t ld_out, hipStream_t s) {
    FftPlan plan;
    if (!make_plan(nt_fft / 2, &plan)) return hipErrorInvalidValue;
    if (nrows <= 0) return hipSuccess;
    const int Nh = plan.n;
    const size_t lds = 2 * (size_t)Nh * sizeof(float2);
    const int pairs_ok = ((ld_in % 2) == 0 && (reinterpret_cast<uintptr_t>(in) % 8) == 0) ? 1 : 0;
    const int vpt = (Nh + kRowThreads - 1) / kRowThreads;
    dim3 grid(row_grid(nrows)), block(kRowThreads);
#define LAR_R2C(V)                                                                           \
    {                                                                                        \
        set_lds(k_r2c_rows<V>, lds);                                                         \
        hipLaunchKernelGGL(k_r2c_rows<V>, grid, block, lds, s, in, ld_in, n_in, nrows, plan, \
                           out, ld_out, pairs_ok);                                           \
    }
    if (vpt <= 4) LAR_R2C(4)
    else if (vpt <= 8) LAR_R2C(8)
    else if (vpt <= 16) LAR_R2C(16)
    else if (vpt <= 32) LAR_R2C(32)
    else return hipErrorInvalidValue;
#undef LAR_R2C
    return hipGetLastError();
}

hipError_t launch_c2r_rows(const float2* in, int64_t ld_in, int nrows, int nt_fft, float* out,
                           int64_t ld_out, int n_out, float scale, hipStream_t s) {
    FftPlan plan;
    if (!make_plan(nt_fft / 2, &plan)) return hipErrorInvalidValue;
    if (nrows <= 0) return hipSuccess;
    const int Nh = plan.n;
    const size_t lds = 2 * (size_t)Nh * sizeof(float2);
    const int pairs_ok = ((ld_out % 2) == 0 && (reinterpret_cast<uintptr_t>(out) % 8) == 0) ? 1 : 0;
    const int vpt = (Nh + kRowThreads - 1) / kRowThreads;
    dim3 grid(row_grid(nrows)), block(kRowThreads);
#define LAR_C2R(V)                                                                          \
    {                                                                                       \
        set_lds(k_c2r_rows<V>, lds);                                                        \
        hipLaunchKernelGGL(k_c2r_rows<V>, grid, block, lds, s, in, ld_in, nrows, plan, out, \
                           ld_out, n_out, scale, pairs_ok);                                 \
    }
    if (vpt <= 4) LAR_C2R(4)
    else if (vpt <= 8) LAR_C2R(8)
    else if (vpt <= 16) LAR_C2R(16)
    else if (vpt <= 32) LAR_C2R(32)
    else return hipErrorInvalidValue;
#undef LAR_C2R
    return hipGetLastError();
}

// ---------------------------------------------------------------- wire pass

static constexpr int kWireThreads = 256;

__device__ __forceinline__ void fill_full_table(float2* t, int n, int tid, int T) {
    for (int i = tid; i < n; i += T) {
        double s, c;
        sincospi(-2.0 * (double)i / (double)n, &s, &c);
        t[i] = make_float2((float)c, (float)s);
    }
}

// One workgroup per tile of C consecutive time-frequency columns.
template <int VPT, int C>
__global__ __launch_bounds__(kWireThreads) void k_wire_fused(
    const float2* __restrict__ S, int64_t ldS, int n_wires, int n_imp, int F, FftPlan plan,
    const float2* __restrict__ R, float2* __restrict__ M, int64_t ldM) {
    extern __shared__ float2 lds[];
    const int Wf = plan.n, tid = threadIdx.x, T = blockDim.x;
    float2* A = lds;               // [Wf][C]
    float2* tw = lds + Wf * C;     // [Wf]
    fill_full_table(tw, Wf, tid, T);
    const TwFull twf{tw};
    const int f0 = xcd_tile(blockIdx.x, gridDim.x) * C;
    const int nel = Wf * C;
    float2 acc[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) acc[i] = make_float2(0.f, 0.f);

    for (int k = 0; k < n_imp; ++k) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            int e = tid + i * T;
            if (e < nel) {
                int p = e / C, c = e % C, f = f0 + c;
                float2 v = make_float2(0.f, 0.f);
                if (p < n_wires && f < F) v = S[(int64_t)(p * n_imp + k) * ldS + f];
                A[e] = v;
            }
        }
        __syncthreads();
        fft_lds<VPT, C>(A, plan, tid, T, twf, false);
        const float2* Rk = R + (int64_t)k * Wf * F;
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            int e = tid + i * T;
            if (e < nel) {
                int p = e / C, c = e % C, f = f0 + c;
                if (f < F) {
                    float2 r = Rk[(int64_t)p * F + f];
                    float2 a = A[e];
                    acc[i].x += a.x * r.x - a.y * r.y;
                    acc[i].y += a.x * r.y + a.y * r.x;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        int e = tid + i * T;
        if (e < nel) A[e] = acc[i];
    }
    __syncthreads();
    fft_lds<VPT, C>(A, plan, tid, T, twf, true);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        int e = tid + i * T;
        if (e < nel) {
            int p = e / C, c = e % C, f = f0 + c;
            if (p < n_wires && f < F) M[(int64_t)p * ldM + f] = A[e];
        }
    }
}

template <int VPT, int C>
static hipError_t wire_launch(const float2* S, int64_t ldS, int n_wires, int n_imp, int F,
                              const FftPlan& plan, const float2* R, float2* M, int64_t ldM,
                              hipStream_t s) {
    const size_t lds = ((size_t)plan.n * C + plan.n) * sizeof(float2);
    set_lds(k_wire_fused<VPT, C>, lds);
    dim3 grid((F + C - 1) / C), block(kWireThreads);
    hipLaunchKernelGGL((k_wire_fused<VPT, C>), grid, block, lds, s, S, ldS, n_wires, n_imp, F,
                       plan, R, M, ldM);
    return hipGetLastError();
}

hipError_t launch_wire_fused(const float2* S, int64_t ldS, int n_wires, int n_imp, int nw_fft,
                             int F, const float2* R, float2* M, int64_t ldM, hipStream_t s) {
    FftPlan plan;
    if (!make_plan(nw_fft, &plan)) return hipErrorInvalidValue;
    if (F <= 0) return hipSuccess;
    // C columns per tile: 16 (128-byte row segments) while the tile fits in
    // 32 values per thread, else 8
    if (nw_fft * 16 <= 8 * kWireThreads)
        return wire_launch<8, 16>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, s);
    if (nw_fft * 16 <= 16 * kWireThreads)
        return wire_launch<16, 16>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, s);
    if (nw_fft * 16 <= 32 * kWireThreads)
        return wire_launch<32, 16>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, s);
    if (nw_fft * 8 <= 32 * kWireThreads)
        return wire_launch<32, 8>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- response spectrum
//
// rows: time spectra [n_imp][nrw][ld_rows] of the response rows (dw = row -
// half_w); resp[k][p][f] = sum over rows with dw mod Wf = p, then a forward
// FFT over p.
template <int VPT, int C>
__global__ __launch_bounds__(kWireThreads) void k_wire_spectrum(
    const float2* __restrict__ rows, int64_t ld_rows, int nrw, int half_w, int F, FftPlan plan,
    float2* __restrict__ resp) {
    extern __shared__ float2 lds[];
    const int Wf = plan.n, tid = threadIdx.x, T = blockDim.x;
    float2* A = lds;
    float2* tw = lds + Wf * C;
    fill_full_table(tw, Wf, tid, T);
    const int k = blockIdx.y;
    const int f0 = blockIdx.x * C;
    const int nel = Wf * C;
    for (int e = tid; e < nel; e += T) A[e] = make_float2(0.f, 0.f);
    __syncthreads();
    // rows sharing a wire index are summed by one thread each, in order
    for (int e = tid; e < nel; e += T) {
        int p = e / C, c = e % C, f = f0 + c;
        if (f >= F) continue;
        float2 a = make_float2(0.f, 0.f);
        for (int i = 0; i < nrw; ++i) {
            int dw = i - half_w;
            int pi = ((dw % Wf) + Wf) % Wf;
            if (pi == p) a = cadd(a, rows[((int64_t)k * nrw + i) * ld_rows + f]);
        }
        A[e] = a;
    }
    __syncthreads();
    fft_lds<VPT, C>(A, plan, tid, T, TwFull{tw}, false);
    for (int e = tid; e < nel; e += T) {
        int p = e / C, c = e % C, f = f0 + c;
        if (f < F) resp[((int64_t)k * Wf + p) * F + f] = A[e];
    }
}

hipError_t launch_wire_spectrum(const float2* rows, int64_t ld_rows, int n_imp, int nrw,
                                int half_w, int nw_fft, int F, float2* resp, hipStream_t s) {
    FftPlan plan;
    if (!make_plan(nw_fft, &plan)) return hipErrorInvalidValue;
    constexpr int C = 8;
    const size_t lds = ((size_t)plan.n * C + plan.n) * sizeof(float2);
    dim3 grid((F + C - 1) / C, n_imp), block(kWireThreads);
    if (nw_fft * C <= 8 * kWireThreads) {
        set_lds(k_wire_spectrum<8, C>, lds);
        hipLaunchKernelGGL((k_wire_spectrum<8, C>), grid, block, lds, s, rows, ld_rows, nrw,
                           half_w, F, plan, resp);
    } else if (nw_fft * C <= 32 * kWireThreads) {
        set_lds(k_wire_spectrum<32, C>, lds);
        hipLaunchKernelGGL((k_wire_spectrum<32, C>), grid, block, lds, s, rows, ld_rows, nrw,
                           half_w, F, plan, resp);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- fill

__global__ void k_fill_zero(float4* __restrict__ p, int64_t n4) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (; i < n4; i += step) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}
__global__ void k_fill_zero_tail(float* __restrict__ p, int64_t n) {
    int64_t i = threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Zero n floats at p (p 16-byte aligned).  A kernel, not a memset node, so
// that it can sit inside a captured graph.
hipError_t launch_fill(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t n4 = n / 4;
    if (n4 > 0) {
        int64_t blocks = (n4 + 255) / 256;
        int64_t cap = 8 * (int64_t)device_cus();
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(blocks < cap ? blocks : cap)), dim3(256),
                           0, s, reinterpret_cast<float4*>(p), n4);
    }
    int64_t tail = n - 4 * n4;
    if (tail > 0) hipLaunchKernelGGL(k_fill_zero_tail, dim3(1), dim3(64), 0, s, p + 4 * n4, tail);
    return hipGetLastError();
}

}  // namespace lar
