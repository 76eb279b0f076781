// raster_kernels.hip -- "Raster" and "Scatter-add" (paper Sec. 2.2) for gfx950.
//
// One workgroup takes a chunk of consecutive depositions (parallel over
// ionization groups, Sec. 2.3).  Per depo: the n-sigma windows on both axes
// (decided in FP64), the 1D Gaussian bin integrals from erfc (FP32), the
// patch q*wt[j]*wx[m] or its fluctuated counts.  Patches of the chunk are
// summed in an LDS tile covering the chunk's bounding box (track depos are
// contiguous, so neighbouring patches overlap heavily) and the tile is
// flushed with one global float atomic per non-zero cell, coalesced along
// ticks.  Chunks whose box does not fit the tile, and depos whose window is
// larger than the per-depo weight slots, add their cells with direct global
// atomics.
//
// Fluctuation (paper Sec. 3.1): per bin, Binomial(rint|q|, p) or
// Poisson(|q| p) with p = wt*wx, uniforms from Philox4x32-10 (Salmon et al.,
// SC'11) keyed by seed and counter (depo, event, bin, plane*2^24 + draw).
// Binomial: inversion for n*min(p,1-p) < 10, BTRD otherwise (Hormann 1993);
// Poisson: inversion for lambda < 10, PTRS otherwise (Hormann 1993).  The
// sampler is FP64 without contraction so that a CPU implementation of the
// same steps makes the same decisions.
#include "lar_internal.hpp"

namespace lar {

// ---------------------------------------------------------------- Philox

struct PhiloxStream {
    uint32_t k0, k1;
    uint32_t c0, c1, c2, c3;
    uint32_t b2, b3;
    int left;
};

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// 52-bit uniform strictly inside (0, 1): ((a>>6) 2^26 + (b>>6) + 1/2) 2^-52.
__device__ __forceinline__ double u52(uint32_t a, uint32_t b) {
#pragma clang fp contract(off)
    double hi = (double)(a >> 6), lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 4503599627370496.0);
}

__device__ __forceinline__ void stream_init(PhiloxStream& s, uint64_t seed, uint32_t depo,
                                            uint32_t event, uint32_t bin, uint32_t plane) {
    s.k0 = (uint32_t)seed;
    s.k1 = (uint32_t)(seed >> 32);
    s.c0 = depo;
    s.c1 = event;
    s.c2 = bin;
    s.c3 = plane << 24;
    s.left = 0;
}

__device__ __forceinline__ double next_uniform(PhiloxStream& s) {
    if (s.left == 0) {
        uint32_t o0 = s.c0, o1 = s.c1, o2 = s.c2, o3 = s.c3;
        philox4x32_10(o0, o1, o2, o3, s.k0, s.k1);
        s.c3 += 1u;
        s.b2 = o2;
        s.b3 = o3;
        s.left = 2;
        return u52(o0, o1);
    }
    s.left = 0;
    return u52(s.b2, s.b3);
}

// ---------------------------------------------------------------- samplers

#define LAR_MAX_TRIES 1000

// log k! - [(k + 1/2) log(k+1) - (k+1) + log(2 pi)/2]
__device__ double stirling_tail(double k) {
#pragma clang fp contract(off)
    if (k < 10.0)
        return lgamma(k + 1.0) - (k + 0.5) * log(k + 1.0) + (k + 1.0) - 0.91893853320467274178;
    double r = 1.0 / (k + 1.0);
    double r2 = r * r;
    return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * r2) * r2) * r;
}

// Binomial by inversion from k = 0 (p <= 1/2, n p < 10).
__device__ double binom_inversion(double n, double p, PhiloxStream& s) {
#pragma clang fp contract(off)
    double q = 1.0 - p;
    double ratio = p / q;
    double g = ratio * (n + 1.0);
    double f0 = exp(n * log1p(-p));
    for (int tries = 0; tries < LAR_MAX_TRIES; ++tries) {
        double u = next_uniform(s);
        double f = f0;
        double k = 0.0;
        for (;;) {
            if (u < f) return k;
            if (k >= n || k > 110.0) break;
            u = u - f;
            k = k + 1.0;
            f = f * (g / k - ratio);
        }
    }
    return floor(n * p);
}

// Binomial by BTRD, transformed rejection with decomposition (p <= 1/2, n p >= 10).
__device__ double binom_btrd(double n, double p, PhiloxStream& s) {
#pragma clang fp contract(off)
    double m = floor((n + 1.0) * p);
    double r = p / (1.0 - p);
    double nr = (n + 1.0) * r;
    double npq = n * p * (1.0 - p);
    double spq = sqrt(npq);
    double b = 1.15 + 2.53 * spq;
    double a = -0.0873 + 0.0248 * b + 0.01 * p;
    double c = n * p + 0.5;
    double alpha = (2.83 + 5.1 / b) * spq;
    double vr = 0.92 - 4.2 / b;
    double urvr = 0.86 * vr;
    for (int tries = 0; tries < LAR_MAX_TRIES; ++tries) {
        double v = next_uniform(s);
        double u;
        if (v <= urvr) {
            u = v / vr - 0.43;
            return floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
        }
        if (v >= vr) {
            u = next_uniform(s) - 0.5;
        } else {
            u = v / vr - 0.93;
            u = copysign(0.5, u) - u;
            v = next_uniform(s) * vr;
        }
        double us = 0.5 - fabs(u);
        double k = floor((2.0 * a / us + b) * u + c);
        if (k < 0.0 || k > n) continue;
        v = v * alpha / (a / (us * us) + b);
        double km = fabs(k - m);
        if (km <= 15.0) {
            double f = 1.0;
            if (m < k) {
                for (double i = m + 1.0; i <= k; i = i + 1.0) f = f * (nr / i - r);
            } else if (m > k) {
                for (double i = k + 1.0; i <= m; i = i + 1.0) v = v * (nr / i - r);
            }
            if (v <= f) return k;
            continue;
        }
        v = log(v);
        double rho = (km / npq) * (((km / 3.0 + 0.625) * km + 1.0 / 6.0) / npq + 0.5);
        double t = -km * km / (2.0 * npq);
        if (v < t - rho) return k;
        if (v > t + rho) continue;
        double nm = n - m + 1.0;
        double h = (m + 0.5) * log((m + 1.0) / (r * nm)) + stirling_tail(m) + stirling_tail(n - m);
        double nk = n - k + 1.0;
        if (v <= h + (n + 1.0) * log(nm / nk) + (k + 0.5) * log(nk * r / (k + 1.0))
                      - stirling_tail(k) - stirling_tail(n - k))
            return k;
    }
    return m;
}

__device__ double sample_binomial(double n, double p, PhiloxStream& s) {
#pragma clang fp contract(off)
    if (!(n > 0.0) || !(p > 0.0)) return 0.0;
    if (p >= 1.0) return n;
    bool flip = p > 0.5;
    double pp = flip ? 1.0 - p : p;
    double k = (n * pp < 10.0) ? binom_inversion(n, pp, s) : binom_btrd(n, pp, s);
    return flip ? n - k : k;
}

__device__ double sample_poisson(double lam, PhiloxStream& s) {
#pragma clang fp contract(off)
    if (!(lam > 0.0)) return 0.0;
    if (lam < 10.0) {
        double p0 = exp(-lam);
        for (int tries = 0; tries < LAR_MAX_TRIES; ++tries) {
            double u = next_uniform(s);
            double p = p0, cdf = p0, k = 0.0;
            while (u > cdf) {
                if (k > 200.0) break;
                k = k + 1.0;
                p = p * lam / k;
                cdf = cdf + p;
            }
            if (u <= cdf) return k;
        }
        return floor(lam);
    }
    double slam = sqrt(lam);
    double loglam = log(lam);
    double b = 0.931 + 2.53 * slam;
    double a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int tries = 0; tries < LAR_MAX_TRIES; ++tries) {
        double u = next_uniform(s) - 0.5;
        double v = next_uniform(s);
        double us = 0.5 - fabs(u);
        double k = floor((2.0 * a / us + b) * u + lam + 0.43);
        if (us >= 0.07 && v <= vr) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        if (log(v) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0))
            return k;
    }
    return floor(lam);
}

// Signed count of one bin.
__device__ __noinline__ float bin_count(int mode, float q, double p, uint64_t seed, uint32_t depo,
                                        uint32_t event, uint32_t bin, uint32_t plane) {
#pragma clang fp contract(off)
    PhiloxStream s;
    stream_init(s, seed, depo, event, bin, plane);
    double aq = fabs((double)q);
    double n = (mode == 1) ? sample_binomial(rint(aq), p, s) : sample_poisson(aq * p, s);
    float r = (float)n;
    return q < 0.f ? -r : r;
}

__global__ void k_sample_counts(int mode, int64_t n, const float* __restrict__ q,
                                const double* __restrict__ p, const uint32_t* __restrict__ ctr3,
                                uint32_t plane, uint64_t seed, float* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = bin_count(mode, q[i], p[i], seed, ctr3[3 * i], ctr3[3 * i + 1], ctr3[3 * i + 2],
                       plane);
}

hipError_t launch_sample_counts(int mode, int64_t n, const float* q, const double* p,
                                const uint32_t* ctr3, uint32_t plane, uint64_t seed, float* out,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mode,
                       n, q, p, ctr3, plane, seed, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- windows

struct Window {
    int lo, n;     // n == 0: no overlap with the grid
    bool point;
};

// Bins of one axis intersecting [mu - ns sigma, mu + ns sigma]; the same FP64
// operation sequence as the definition so that integer decisions agree
// exactly with any other IEEE implementation of it.
__device__ __forceinline__ Window axis_window(double mu, double sg, double ns, double org,
                                              double wd, int nbins) {
#pragma clang fp contract(off)
    Window w{0, 0, false};
    if (sg < 1e-6 * wd) {
        double f = floor((mu - org) / wd);
        if (!(f >= 0.0) || f >= (double)nbins) return w;
        w.lo = (int)f;
        w.n = 1;
        w.point = true;
        return w;
    }
    double flo = floor((mu - ns * sg - org) / wd);
    double fhi = floor((mu + ns * sg - org) / wd);
    if (flo < 0.0) flo = 0.0;
    if (fhi > (double)(nbins - 1)) fhi = (double)(nbins - 1);
    if (!(flo <= fhi)) return w;
    w.lo = (int)flo;
    w.n = (int)fhi - w.lo + 1;
    return w;
}

// Tail mass of the standard normal beyond |z|.
__device__ __forceinline__ float normal_tail(float z) {
    return 0.5f * erfcf(fabsf(z) * 0.70710678118654752f);
}

// Edge e's standardized coordinate (FP64 subtraction, then FP32).
__device__ __forceinline__ float edge_z(double org, double wd, int e, double mu, double inv_sg) {
    return (float)((org + (double)e * wd - mu) * inv_sg);
}

// Phi(zb) - Phi(za) from the two tail masses.
__device__ __forceinline__ float bin_weight(float za, float zb, float ta, float tb) {
    if (za >= 0.f) return ta - tb;
    if (zb <= 0.f) return tb - ta;
    return 1.f - ta - tb;
}

// Weights of n bins starting at lo into w[stride * i].
__device__ void axis_weights(double mu, double sg, double org, double wd, const Window& win,
                             float* w, int stride) {
    if (win.point) {
        w[0] = 1.f;
        return;
    }
    double inv = 1.0 / sg;
    float za = edge_z(org, wd, win.lo, mu, inv);
    float ta = normal_tail(za);
    for (int i = 0; i < win.n; ++i) {
        float zb = edge_z(org, wd, win.lo + i + 1, mu, inv);
        float tb = normal_tail(zb);
        w[i * stride] = bin_weight(za, zb, ta, tb);
        za = zb;
        ta = tb;
    }
}

// Weight of a single bin (slow path for depos with large windows).
__device__ __forceinline__ float single_weight(double mu, double sg, double org, double wd,
                                               const Window& win, int i) {
    if (win.point) return 1.f;
    double inv = 1.0 / sg;
    float za = edge_z(org, wd, win.lo + i, mu, inv);
    float zb = edge_z(org, wd, win.lo + i + 1, mu, inv);
    return bin_weight(za, zb, normal_tail(za), normal_tail(zb));
}

// ---------------------------------------------------------------- raster kernel

static constexpr int kRasterThreads = 256;
static constexpr int kChunk = 128;        // depos per chunk
static constexpr int kMaxT = 16;          // regular window limits (bins)
static constexpr int kMaxX = 32;
static constexpr int kSlot = kMaxT + kMaxX + 1;   // +1 pad against LDS bank conflicts
static constexpr int kTileCap = 8192;     // LDS tile (floats)

__device__ __forceinline__ bool depo_finite(float a, float b, float c, float d, float e) {
    return isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d) && isfinite(e);
}

template <bool FLUCT>
__device__ __forceinline__ float cell_value(const RasterArgs& A, float q, float wt, float wx,
                                            uint32_t depo, int m, int j) {
    if (!FLUCT) return q * wt * wx;
    double p = (double)(wt * wx);
    uint32_t bin = (uint32_t)((int64_t)m * A.n_ticks + j);
    return bin_count(A.mode, q, p, A.seed, depo, A.event, bin, A.plane);
}

template <bool FLUCT>
__global__ __launch_bounds__(kRasterThreads) void k_raster(RasterArgs A, const float* __restrict__ Q,
                                                           const float* __restrict__ Tm,
                                                           const float* __restrict__ X,
                                                           const float* __restrict__ ST,
                                                           const float* __restrict__ SX, int64_t n,
                                                           float* __restrict__ grid) {
    __shared__ float s_w[kChunk * kSlot];
    __shared__ float s_tile[kTileCap];
    __shared__ int s_jlo[kChunk], s_nt[kChunk], s_mlo[kChunk], s_nx[kChunk];
    __shared__ float s_q[kChunk];
    __shared__ int s_off[kChunk + 1];
    __shared__ int s_big[kChunk];
    __shared__ int s_nbig;
    __shared__ int s_box[4];   // jmin, jmax, mmin, mmax
    __shared__ int s_wsum[kRasterThreads / 64];

    const int tid = threadIdx.x;
    for (int i = tid; i < kTileCap; i += kRasterThreads) s_tile[i] = 0.f;
    const int64_t nchunks = (n + kChunk - 1) / kChunk;

    for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        const int64_t base = chunk * kChunk;
        if (tid == 0) {
            s_nbig = 0;
            s_box[0] = INT_MAX; s_box[1] = INT_MIN; s_box[2] = INT_MAX; s_box[3] = INT_MIN;
        }
        __syncthreads();
        // ---- windows (one thread per depo)
        int cells = 0;
        if (tid < kChunk) {
            int64_t d = base + tid;
            int nt = 0, nx = 0, jlo = 0, mlo = 0;
            float q = 0.f;
            if (d < n) {
                q = Q[d];
                float t = Tm[d], x = X[d], st = ST[d], sx = SX[d];
                if (depo_finite(q, t, x, st, sx)) {
                    Window wt = axis_window(t, st, A.nsig, A.org_t, A.wd_t, A.n_ticks);
                    Window wx = wt.n ? axis_window(x, sx, A.nsig, A.org_x, A.wd_x, A.n_rows)
                                     : Window{0, 0, false};
                    if (wt.n && wx.n) {
                        nt = wt.n; nx = wx.n; jlo = wt.lo; mlo = wx.lo;
                        if (wt.point) nt = -nt;   // sign marks a point axis (weights skip erfc)
                        if (wx.point) nx = -nx;
                    }
                }
            }
            int ant = abs(nt), anx = abs(nx);
            bool regular = ant > 0 && ant <= kMaxT && anx <= kMaxX;
            if (ant > 0 && !regular) {
                int slot = atomicAdd(&s_nbig, 1);
                s_big[slot] = tid;
            }
            s_jlo[tid] = jlo; s_mlo[tid] = mlo; s_nt[tid] = nt; s_nx[tid] = nx; s_q[tid] = q;
            cells = regular ? ant * anx : 0;
            if (regular) {
                atomicMin(&s_box[0], jlo); atomicMax(&s_box[1], jlo + ant - 1);
                atomicMin(&s_box[2], mlo); atomicMax(&s_box[3], mlo + anx - 1);
            }
        }
        // ---- exclusive scan of cell counts (threads >= kChunk contribute 0)
        {
            int lane = tid & 63, wv = tid >> 6;
            int v = cells;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                int u = __shfl_up(v, o, 64);
                if (lane >= o) v += u;
            }
            if (lane == 63) s_wsum[wv] = v;
            __syncthreads();
            int add = 0;
            for (int i = 0; i < wv; ++i) add += s_wsum[i];
            if (tid < kChunk) s_off[tid] = add + v - cells;
            if (tid == kChunk - 1) s_off[kChunk] = add + v;
        }
        __syncthreads();
        // ---- 1D weights: two threads per depo (time axis, pitch axis)
        {
            int d = tid >> 1, ax = tid & 1;
            int64_t gd = base + d;
            int nt = s_nt[d], nx = s_nx[d];
            int ant = abs(nt), anx = abs(nx);
            if (gd < n && ant > 0 && ant <= kMaxT && anx <= kMaxX) {
                float* w = s_w + d * kSlot;
                if (ax == 0) {
                    Window win{s_jlo[d], ant, nt < 0};
                    axis_weights(Tm[gd], ST[gd], A.org_t, A.wd_t, win, w, 1);
                } else {
                    Window win{s_mlo[d], anx, nx < 0};
                    axis_weights(X[gd], SX[gd], A.org_x, A.wd_x, win, w + kMaxT, 1);
                }
            }
        }
        __syncthreads();
        // ---- cells
        const int total = s_off[kChunk];
        const int jmin = s_box[0], mmin = s_box[2];
        const int span_t = s_box[1] - jmin + 1, span_x = s_box[3] - mmin + 1;
        const bool use_tile = total > 0 && (int64_t)span_t * span_x <= kTileCap;
        {
            int d = 0;
            for (int c = tid; c < total; c += kRasterThreads) {
                while (s_off[d + 1] <= c) ++d;
                int ant = abs(s_nt[d]);
                int local = c - s_off[d];
                int a = local / ant, b = local - a * ant;
                const float* w = s_w + d * kSlot;
                int j = s_jlo[d] + b, m = s_mlo[d] + a;
                float v = cell_value<FLUCT>(A, s_q[d], w[b], w[kMaxT + a], (uint32_t)(base + d), m, j);
                if (v != 0.f) {
                    if (use_tile)
                        atomicAdd(&s_tile[(m - mmin) * span_t + (j - jmin)], v);
                    else
                        atomicAdd(&grid[(int64_t)m * A.ld + j], v);
                }
            }
        }
        __syncthreads();
        // ---- flush the tile (one atomic per non-zero cell), leave it zeroed
        if (use_tile) {
            const int area = span_t * span_x;
            for (int e = tid; e < area; e += kRasterThreads) {
                float v = s_tile[e];
                if (v != 0.f) {
                    int r = e / span_t, cidx = e - r * span_t;
                    atomicAdd(&grid[(int64_t)(mmin + r) * A.ld + jmin + cidx], v);
                    s_tile[e] = 0.f;
                }
            }
        }
        // ---- depos with windows beyond the slots: all threads, per cell
        const int nbig = s_nbig;
        for (int bi = 0; bi < nbig; ++bi) {
            int d = s_big[bi];
            int64_t gd = base + d;
            int nt = s_nt[d], nx = s_nx[d];
            int ant = abs(nt), anx = abs(nx);
            Window wt{s_jlo[d], ant, nt < 0}, wx{s_mlo[d], anx, nx < 0};
            float t = Tm[gd], st = ST[gd], x = X[gd], sx = SX[gd], q = s_q[d];
            int64_t ncell = (int64_t)ant * anx;
            for (int64_t c = tid; c < ncell; c += kRasterThreads) {
                int a = (int)(c / ant), b = (int)(c - (int64_t)a * ant);
                float wtv = single_weight(t, st, A.org_t, A.wd_t, wt, b);
                float wxv = single_weight(x, sx, A.org_x, A.wd_x, wx, a);
                int j = wt.lo + b, m = wx.lo + a;
                float v = cell_value<FLUCT>(A, q, wtv, wxv, (uint32_t)gd, m, j);
                if (v != 0.f) atomicAdd(&grid[(int64_t)m * A.ld + j], v);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_raster(const RasterArgs& a, const float* q, const float* t, const float* x,
                         const float* st, const float* sx, int64_t n, float* grid, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nchunks = (n + kChunk - 1) / kChunk;
    int64_t cap = 8 * (int64_t)device_cus();
    dim3 grd((unsigned)(nchunks < cap ? nchunks : cap)), blk(kRasterThreads);
    if (a.mode == 0)
        hipLaunchKernelGGL(k_raster<false>, grd, blk, 0, s, a, q, t, x, st, sx, n, grid);
    else
        hipLaunchKernelGGL(k_raster<true>, grd, blk, 0, s, a, q, t, x, st, sx, n, grid);
    return hipGetLastError();
}

}  // namespace lar
