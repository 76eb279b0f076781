// lar_internal.hpp -- device helpers and launcher declarations of the gfx950
// LArTPC signal-simulation library.  Not part of the public ABI (lar.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lar.h"

namespace lar {

// ---------------------------------------------------------------- FFT plan
//
// Mixed-radix Stockham autosort FFT (Stockham 1966; the formulation of Van
// Loan, "Computational Frameworks for the FFT", 1992): pass p with radix R
// and sub-transform size Ns (product of earlier radices) reads the R inputs
// of butterfly j at stride n/R, applies the twiddles exp(-+2 pi i r (j mod Ns)
// / (Ns R)), and writes the R outputs at (j div Ns) Ns R + (j mod Ns) + r Ns.
// Lengths are 2^a 3^b with passes of radix 8, 4, 3 and 2; the order of the
// passes is a schedule choice (make_plan's `order`).
constexpr int kMaxPasses = 16;
constexpr size_t kLdsBytes = 160 * 1024;   // LDS of one gfx950 compute unit
constexpr int kPlanOrders = 6;

struct FftPlan {
    int n;
    int npass;
    int radix[kMaxPasses];
};

// Host: build the plan for length n; false if n is not 2^a 3^b (n >= 1).
// order 0: radix 8 passes first, then one 4 or 2, then the 3s; 1: radix 4
// passes, then 3s, then one 2 (no radix 8); 2: 3s first, then 8s, then
// 4/2; 3: the reverse of order 0; 4: radix 8 passes first, then each
// remaining factor 2 paired with a 3 as a radix-6 pass, then what is left
// (fewer passes when both 2 and 3 remain).
bool make_plan(int n, FftPlan* plan, int order = 0);

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Workgroup barrier that orders LDS only: outstanding global loads and
// atomics are not waited for (a plain __syncthreads also fences global
// memory, which stalls on in-flight prefetches and fire-and-forget atomics).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Small DFTs, sign -1 (forward) or +1 (inverse) in the exponent.
template <int R>
__device__ __forceinline__ void dft_small(float2* v, bool inv);

template <>
__device__ __forceinline__ void dft_small<2>(float2* v, bool) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft_small<3>(float2* v, bool inv) {
    const float s3 = 0.86602540378443865f;   // sin(2 pi / 3)
    float2 t1 = cadd(v[1], v[2]);
    float2 d = csub(v[1], v[2]);
    float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    // forward: y1 = t2 - i s3 d, y2 = t2 + i s3 d; inverse swaps the signs
    float sx = inv ? -s3 : s3;
    float2 id = make_float2(sx * d.y, -sx * d.x);   // -i * sx * d
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, id);
    v[2] = csub(t2, id);
}

template <>
__device__ __forceinline__ void dft_small<4>(float2* v, bool inv) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    // forward: y1 = a1 - i b1, y3 = a1 + i b1
    float2 mib1 = inv ? make_float2(-b1.y, b1.x) : make_float2(b1.y, -b1.x);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, mib1);
    v[3] = csub(a1, mib1);
}

template <>
__device__ __forceinline__ void dft_small<8>(float2* v, bool inv) {
    // two 4-point DFTs of the even and odd samples, combined with W8^k
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<4>(e, inv);
    dft_small<4>(o, inv);
    const float c = 0.70710678118654752f;
    const float sg = inv ? 1.f : -1.f;   // W8 = exp(sg i pi/4)
    float2 w1 = cmul(o[1], make_float2(c, sg * c));
    float2 w2 = make_float2(-sg * o[2].y, sg * o[2].x);     // * exp(sg i pi/2) = sg i
    float2 w3 = cmul(o[3], make_float2(-c, sg * c));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], w1);
    v[5] = csub(e[1], w1);
    v[2] = cadd(e[2], w2);
    v[6] = csub(e[2], w2);
    v[3] = cadd(e[3], w3);
    v[7] = csub(e[3], w3);
}

// 6-point DFT as 2 x 3: E = DFT3(x0, x2, x4), O = DFT3(x1, x3, x5), then
// X[k] = E[k] + W6^k O[k] and X[k+3] = E[k] - W6^k O[k] (W6 = exp(-+2 pi i / 6)).
template <>
__device__ __forceinline__ void dft_small<6>(float2* v, bool inv) {
    float2 e[3] = {v[0], v[2], v[4]};
    float2 o[3] = {v[1], v[3], v[5]};
    dft_small<3>(e, inv);
    dft_small<3>(o, inv);
    const float s3 = 0.86602540378443865f;
    const float sg = inv ? 1.f : -1.f;
    const float2 w1 = cmul(o[1], make_float2(0.5f, sg * s3));
    const float2 w2 = cmul(o[2], make_float2(-0.5f, sg * s3));
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], w1);
    v[4] = csub(e[1], w1);
    v[2] = cadd(e[2], w2);
    v[5] = csub(e[2], w2);
}

// Twiddle accessors: tw(m) = exp(-2 pi i m / n) for 0 <= m < n.
struct TwFull {           // table of n entries
    const float2* t;
    __device__ __forceinline__ float2 operator()(int m) const { return t[m]; }
};
struct TwHalf {           // table h[k] = exp(-pi i k / n), k < n (half-angle table)
    const float2* t;
    int n;
    __device__ __forceinline__ float2 operator()(int m) const {   // branch-free
        const int i = 2 * m;
        const bool hi = i >= n;
        const float2 v = t[hi ? i - n : i];
        return hi ? make_float2(-v.x, -v.y) : v;
    }
};

// One Stockham pass over NS interleaved sequences held in LDS (element i of
// sequence s at A[i*NS + s]).  All loads of a thread happen before the
// barrier and all stores after it, so the pass is in place.
template <int R, int MAXB, int NS, class TW>
__device__ __forceinline__ void stockham_pass(float2* A, int n, int Ns, int tid, int T,
                                              const TW& tw, bool inv) {
    const int nb = n / R;
    const int total = nb * NS;
    const int stride = n / (Ns * R);
    // Ns is a power of two in every pass before the first radix-3 one
    // (wave-uniform test): a mask then replaces the integer remainder
    const bool ns_pow2 = (Ns & (Ns - 1)) == 0;
    float2 v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        int w = tid + b * T;
        dst[b] = -1;
        if (w < total) {
            int s = w % NS, j = w / NS;
            int k = ns_pow2 ? (j & (Ns - 1)) : j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = A[(j + r * nb) * NS + s];
                if (r > 0) {
                    float2 t = tw(r * k * stride);
                    x = inv ? cmulc(x, t) : cmul(x, t);
                }
                v[b][r] = x;
            }
            dst[b] = ((j - k) * R + k) * NS + s;
        }
    }
    lds_barrier();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (dst[b] >= 0) {
            dft_small<R>(v[b], inv);
#pragma unroll
            for (int r = 0; r < R; ++r) A[dst[b] + r * Ns * NS] = v[b][r];
        }
    }
    lds_barrier();
}

// ---- transforms with pass-major twiddle tables and optional LDS padding
//
// LDS index with one float2 of padding after every 32 (PAD): the strided
// writes of the first Stockham passes (stride R elements between lanes)
// then spread over the LDS banks.
template <int PAD>
__device__ __forceinline__ int lidx(int i) { return PAD ? i + (i >> 5) : i; }
// float2 slots of an n-element padded buffer
__host__ __device__ inline int lds_slots(int n, int pad) { return pad ? n + (n >> 5) + 1 : n; }

// stockham_pass of one sequence in a padded LDS buffer (lidx<1>).
template <int R, int MAXB, class TW>
__device__ __forceinline__ void stockham_pass_tw(float2* A, int n, int Ns, int tid, int T, const TW& tw, bool inv) {
    const int nb = n / R;
    const int stride = n / (Ns * R);
    const bool ns_pow2 = (Ns & (Ns - 1)) == 0;
    float2 v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int j = tid + b * T;
        dst[b] = -1;
        if (j < nb) {
            const int k = ns_pow2 ? (j & (Ns - 1)) : j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = A[lidx<1>(j + r * nb)];
                if (r > 0) {
                    const float2 t = tw(r * k * stride);
                    x = inv ? cmulc(x, t) : cmul(x, t);
                }
                v[b][r] = x;
            }
            dst[b] = (j - k) * R + k;
        }
    }
    lds_barrier();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (dst[b] >= 0) {
            dft_small<R>(v[b], inv);
#pragma unroll
            for (int r = 0; r < R; ++r) A[lidx<1>(dst[b] + r * Ns)] = v[b][r];
        }
    }
    lds_barrier();
}

// Full transform of NS interleaved length-n sequences in LDS by T threads,
// VPT >= n*NS/T values per thread.  Unnormalised; inv selects exp(+...).
// Plans of radices 8, 4, 3 and 2 only (make_plan orders 0..3).
template <int VPT, int NS, class TW>
__device__ __forceinline__ void fft_lds(float2* A, const FftPlan& plan, int tid, int T,
                                        const TW& tw, bool inv) {
    int Ns = 1;
    for (int p = 0; p < plan.npass; ++p) {
        int R = plan.radix[p];
        if (R == 8)
            stockham_pass<8, (VPT + 7) / 8, NS>(A, plan.n, Ns, tid, T, tw, inv);
        else if (R == 4)
            stockham_pass<4, (VPT + 3) / 4, NS>(A, plan.n, Ns, tid, T, tw, inv);
        else if (R == 3)
            stockham_pass<3, (VPT + 2) / 3, NS>(A, plan.n, Ns, tid, T, tw, inv);
        else
            stockham_pass<2, (VPT + 1) / 2, NS>(A, plan.n, Ns, tid, T, tw, inv);
        Ns *= R;
    }
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit multiplies with the published multipliers and Weyl key
// increments, counter (c0..c3) replaced by the output block.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
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


// Pass-major twiddle tables: pass p (radix R, sub-transform size Ns) owns
// Ns (R - 1) consecutive entries, entry k (R - 1) + r - 1 = exp(-2 pi i r k
// stride / n) with stride = n / (Ns R), so a butterfly reads its R - 1
// twiddles from consecutive slots with no index arithmetic.
__host__ __device__ inline int pm_entries(const FftPlan& plan) {
    int Ns = 1, e = 0;
    for (int p = 0; p < plan.npass; ++p) {
        e += Ns * (plan.radix[p] - 1);
        Ns *= plan.radix[p];
    }
    return e;
}

template <class TW>
__device__ __forceinline__ void build_pm(float2* tp, const FftPlan& plan, const TW& tw, int tid, int T) {
    int Ns = 1, off = 0;
    for (int p = 0; p < plan.npass; ++p) {
        const int R = plan.radix[p], cnt = Ns * (R - 1), stride = plan.n / (Ns * R);
        for (int e = tid; e < cnt; e += T) {
            const int k = e / (R - 1), r = e - k * (R - 1) + 1;
            tp[off + e] = tw(r * k * stride);
        }
        off += cnt;
        Ns *= R;
    }
}

// One Stockham pass as stockham_pass, twiddles from the pass's table tp.
template <int R, int MAXB, int NS, int PAD>
__device__ __forceinline__ void stockham_pass_pm(float2* A, int n, int Ns, int tid, int T, const float2* tp,
                                                 bool inv) {
    const int nb = n / R;
    const int total = nb * NS;
    const bool ns_pow2 = (Ns & (Ns - 1)) == 0;
    float2 v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int w = tid + b * T;
        dst[b] = -1;
        if (w < total) {
            const int s = w % NS, j = w / NS;
            const int k = ns_pow2 ? (j & (Ns - 1)) : j % Ns;
            const float2* t = tp + k * (R - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = A[lidx<PAD>((j + r * nb) * NS + s)];
                if (r > 0) x = inv ? cmulc(x, t[r - 1]) : cmul(x, t[r - 1]);
                v[b][r] = x;
            }
            dst[b] = ((j - k) * R + k) * NS + s;
        }
    }
    lds_barrier();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (dst[b] >= 0) {
            dft_small<R>(v[b], inv);
#pragma unroll
            for (int r = 0; r < R; ++r) A[lidx<PAD>(dst[b] + r * Ns * NS)] = v[b][r];
        }
    }
    lds_barrier();
}

// Passes p0.. of a transform of NS interleaved sequences (as fft_lds),
// with the pass-major tables tp of build_pm (passes before p0 were done
// elsewhere, e.g. in registers).  R6: the plan may hold radix-6 passes
// (without it the radix-6 case is not compiled in, which keeps the
// registers of the other passes' kernels down).
template <int VPT, int NS, int PAD, bool R6 = true>
__device__ __forceinline__ void fft_lds_pm(float2* A, const FftPlan& plan, int tid, int T, const float2* tp,
                                           bool inv, int p0 = 0) {
    int Ns = 1;
    for (int p = 0; p < p0; ++p) {
        tp += Ns * (plan.radix[p] - 1);
        Ns *= plan.radix[p];
    }
    for (int p = p0; p < plan.npass; ++p) {
        const int R = plan.radix[p];
        if (R == 8)
            stockham_pass_pm<8, (VPT + 7) / 8, NS, PAD>(A, plan.n, Ns, tid, T, tp, inv);
        else if (R6 && R == 6)
            stockham_pass_pm<6, (VPT + 5) / 6, NS, PAD>(A, plan.n, Ns, tid, T, tp, inv);
        else if (R == 4)
            stockham_pass_pm<4, (VPT + 3) / 4, NS, PAD>(A, plan.n, Ns, tid, T, tp, inv);
        else if (R == 3)
            stockham_pass_pm<3, (VPT + 2) / 3, NS, PAD>(A, plan.n, Ns, tid, T, tp, inv);
        else
            stockham_pass_pm<2, (VPT + 1) / 2, NS, PAD>(A, plan.n, Ns, tid, T, tp, inv);
        tp += Ns * (R - 1);
        Ns *= R;
    }
}

template <int... Rs>
struct RadixList {};
template <int... Rs>
struct RadixProd {
    static constexpr int v = 1;
};
template <int R, int... Rs>
struct RadixProd<R, Rs...> {
    static constexpr int v = R * RadixProd<Rs...>::v;
};
// entries of the pass-major table taken by passes of radices Rs from Ns = NS on
template <int NS, int... Rs>
struct TableSpan {
    static constexpr int v = 0;
};
template <int NS, int R, int... Rs>
struct TableSpan<NS, R, Rs...> {
    static constexpr int v = NS * (R - 1) + TableSpan<NS * R, Rs...>::v;
};

// One in-place Stockham pass (radix R, sub-transform size NS) of a single
// N-point sequence in the padded A by NT threads, all indices and strides
// compile-time: every butterfly's inputs are read, a barrier, its outputs
// written, a barrier.
template <int N, int NT, int NS, int R>
__device__ __forceinline__ void inplace_pass(float2* A, const float2* __restrict__ tw, int tid, bool inv) {
    constexpr int NB = N / R, MAXB = (NB + NT - 1) / NT;
    float2 x[MAXB][R];
    int ob[MAXB];
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int b = tid + m * NT;
        ob[m] = -1;
        if (NB % NT == 0 || b < NB) {
            const int k = b % NS, li = lidx<1>(b);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // (when NB is a multiple of 32 the pad advances by exactly NB / 32)
                float2 y = A[NB % 32 == 0 ? li + r * (NB + NB / 32) : lidx<1>(b + r * NB)];
                if (r > 0) y = inv ? cmulc(y, tw[k * (R - 1) + r - 1]) : cmul(y, tw[k * (R - 1) + r - 1]);
                x[m][r] = y;
            }
            ob[m] = (b - k) * R + k;
        }
    }
    lds_barrier();
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        if (NB % NT == 0 || ob[m] >= 0) {
            dft_small<R>(x[m], inv);
            const int lo = lidx<1>(ob[m]);
#pragma unroll
            for (int r = 0; r < R; ++r) A[NS % 32 == 0 ? lo + r * (NS + NS / 32) : lidx<1>(ob[m] + r * NS)] = x[m][r];
        }
    }
    lds_barrier();
}

// The passes Rs... of an N-point transform in A from sub-transform size NS
// on (the passes before were done elsewhere), twiddles at tp + TOFF.
template <int N, int NT, int NS, int TOFF>
__device__ __forceinline__ void inplace_passes(RadixList<>, float2*, const float2*, int, bool) {}
template <int N, int NT, int NS, int TOFF, int R, int... Rest>
__device__ __forceinline__ void inplace_passes(RadixList<R, Rest...>, float2* A, const float2* tp, int tid, bool inv) {
    inplace_pass<N, NT, NS, R>(A, tp + TOFF, tid, inv);
    inplace_passes<N, NT, NS * R, TOFF + NS * (R - 1)>(RadixList<Rest...>{}, A, tp, tid, inv);
}

// A row transform with its plan fixed at compile time, for the row kernels:
// the passes Rs... from sub-transform size NS0 (and table entry TOFF0) on.
template <int N, int NT, int NS0, int TOFF0, int... Rs>
struct InplaceRowFft {
    __device__ static void run(float2* A, const float2* tp, int tid, bool inv) {
        inplace_passes<N, NT, NS0, TOFF0>(RadixList<Rs...>{}, A, tp, tid, inv);
    }
};

// blockIdx -> tile with consecutive tiles on one XCD (workgroups are dealt
// round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_tile(int b, int G) {
    int x = b & 7, idx = b >> 3;
    int per = G >> 3, rem = G & 7;
    return x * per + min(x, rem) + idx;
}

// (tile, item) of the linear block index lin over ntiles column tiles of C
// complex columns by nitem items (a batch's items, or item groups).  The
// tiles whose row segments share one 128-byte line (16 / C of them) come
// next to each other for one item, then the same tiles for the next item,
// then the next group of tiles: consecutive indices run together on one XCD
// (xcd_tile), so each line of an item's rows is fetched once for all the
// tiles that use it, and a tile group's response slabs are read from that
// XCD's L2 by every item.  (With the items of one tile next to each other
// instead, a line came back from HBM once per tile that used it: with
// 4-column tiles the batched pass fetched its grid spectra four times.)
__device__ __forceinline__ void tile_item(int lin, int ntiles, int nitem, int C, int& tile, int& item) {
    const int gt = C >= 16 ? 1 : 16 / C;
    const int full = ntiles / gt;
    const int lfull = full * gt * nitem;
    if (lin < lfull) {
        const int grp = lin / (gt * nitem), rem = lin - grp * gt * nitem;
        item = rem / gt;
        tile = grp * gt + (rem - item * gt);
    } else {   // the last, partial group of tiles
        const int r = ntiles - full * gt, rem = lin - lfull;
        item = rem / r;
        tile = full * gt + (rem - item * r);
    }
}

// ---------------------------------------------------------------- launchers
int device_cus();   // compute units of the current device (cached)

// FFT-convolution launch schedule (tunable per plane shape; 0 = default):
// threads per time-axis row workgroup and radix order of the Tf/2 plan,
// columns and threads per wire-pass workgroup and radix order of the Wf plan.
struct Sched {
    int row_threads, row_order;
    int wire_cols, wire_threads, wire_order;
    int raster_tile;   // floats of a raster wave's private LDS tile
};
constexpr int kRasterTileDefault = 512;
bool raster_tile_ok(int tile);   // 384, 512, 640 or 768
int default_row_threads(int nt_fft);
int default_wire_cols(int nw_fft);
int default_wire_threads(int nw_fft);
int default_wire_order(int nw_fft);
bool row_sched_ok(int nt_fft, int threads, int order);
bool wire_sched_ok(int nw_fft, int cols, int threads, int order);
// The schedule registered for this plane shape, else the default one.
Sched sched_for(int n_wires, int n_imp, int n_ticks, int nt_fft, int nw_fft);

// row_in (device, optional): input offset of each row (else row * ld_in);
// the pair loads then need every offset even (row_in_even).
hipError_t launch_r2c_rows(const float* in, int64_t ld_in, int n_in, int nrows, int nt_fft,
                           float2* out, int64_t ld_out, hipStream_t s, int threads = 0,
                           int order = 0, const int64_t* row_in = nullptr, bool row_in_even = false);
// row_off (device, optional): output offset of each row (else row * ld_out);
// the even-pair stores then need every offset even.
hipError_t launch_c2r_rows(const float2* in, int64_t ld_in, int nrows, int nt_fft, float* out,
                           int64_t ld_out, int n_out, float scale, hipStream_t s,
                           const int64_t* row_off = nullptr, bool row_off_even = false,
                           int threads = 0, int order = 0);
// batch > 1: items at S + y * strideS -> M + y * strideM sharing R.
hipError_t launch_wire_fused(const float2* S, int64_t ldS, int n_wires, int n_imp, int nw_fft,
                             int F, const float2* R, float2* M, int64_t ldM, hipStream_t s,
                             int batch = 1, int64_t strideS = 0, int64_t strideM = 0, int cols = 0,
                             int threads = 0, int order = 0);
hipError_t launch_wire_spectrum(const float2* rows, int64_t ld_rows, int n_imp, int nrw,
                                int half_w, int nw_fft, int F, float2* resp, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, hipStream_t s);

struct RasterArgs {
    int n_ticks, n_rows;
    int64_t ld;
    double org_t, wd_t, org_x, wd_x, nsig;
    int mode;
    uint32_t event, plane;
    uint64_t seed;
};
// One raster work item: a depo set rasterized into one plane grid.
// sub_begin is the global index of its first sub-chunk when several items
// are rasterized by one launch (items sorted by sub_begin).
struct RasterItem {
    RasterArgs A;
    const float *q, *t, *x, *st, *sx;
    float* grid;
    int64_t n;
    int64_t sub_begin;
};

// Fluctuated rasters need a workspace: raster_ws_fixed_subs(total
// sub-chunks) bytes of header and sub-chunk flags, then a queue of
// kDeferredBytes-byte deferred bins (capacity = the remaining bytes /
// kDeferredBytes; any capacity, zero included, gives the same result).  The
// mean raster needs none.
constexpr int kRasterSub = 16;   // depos per sub-chunk (one wave's unit of raster work)
__host__ __device__ inline int64_t raster_subchunks(int64_t n) { return (n + kRasterSub - 1) / kRasterSub; }
size_t raster_ws_fixed_subs(int64_t nsub);
size_t raster_ws_fixed(int64_t n);
constexpr size_t kDeferredBytes = 16;
// main_done (optional): recorded on s right after the main raster kernel.
hipError_t launch_raster(const RasterArgs& a, const float* q, const float* t, const float* x,
                         const float* st, const float* sx, int64_t n, float* grid, void* ws,
                         size_t ws_bytes, hipStream_t s, hipEvent_t main_done = nullptr,
                         int tile = kRasterTileDefault);
// items: device table (n_items entries) or nullptr with `one` used alone.
// tile: floats of a wave's LDS tile (raster_tile_ok; the sub-chunks whose
// bounding box exceeds it add straight to the grid).
hipError_t launch_raster_items(int mode, const RasterItem& one, const RasterItem* items, int n_items,
                               int64_t total_sub, void* ws, size_t ws_bytes, hipStream_t s,
                               hipEvent_t main_done = nullptr, int tile = kRasterTileDefault);
// *count (device) = the number of depos with a non-finite field.
hipError_t launch_count_nonfinite(const float* q, const float* t, const float* x, const float* st,
                                  const float* sx, int64_t n, int64_t* count, hipStream_t s);
hipError_t launch_raster_bwd(const RasterArgs& a, const float* q, const float* t, const float* x,
                             const float* st, const float* sx, int64_t n, const float* grid_grad,
                             float* dq, float* dt, float* dx, float* dst, float* dsx, hipStream_t s);
// accumulate: dR += the gradient (else dR = the gradient).
// The grid-gradient spectrum goes to O (which may be S).
hipError_t launch_wire_adjoint(const float2* Gt, int64_t ldG, const float2* S, int64_t ldS, float2* O,
                               int64_t ldO, int n_wires, int n_imp, int nw_fft, int nt_fft,
                               const float2* R, float2* dR, bool want_grid, float resp_scale,
                               hipStream_t s, bool accumulate = true);
// Drift stage: parameters widened to double, plane projections
// (cos, sin, offset) of up to kDriftMaxPlanes planes.
constexpr int kDriftMaxPlanes = 8;
constexpr int kDriftMaxBlocks = 2048;   // grid cap (and partial rows) of the drift kernels
struct DriftConst {
    double v, DL, DT, tau;
    int n_planes;
    double proj[kDriftMaxPlanes][3];
};
hipError_t launch_drift(const DriftConst& C, const float* q0, const float* t0, const float* xd,
                        const float* y, const float* z, int64_t n, float* q, float* t, float* st,
                        float* sx, float* x, hipStream_t s);
// part: kDriftMaxBlocks * 4 doubles of scratch (used when dparams is given).
hipError_t launch_drift_bwd(const DriftConst& C, const float* q0, const float* xd, int64_t n,
                            const float* gq, const float* gt, const float* gst, const float* gsx,
                            const float* gx, float* dq0, float* dt0, float* dxd, float* dy, float* dz,
                            float* dparams, double* part, hipStream_t s);
hipError_t launch_noise_spectrum(const float* amp, int F, int n_wires, uint64_t seed, uint32_t event,
                                 uint32_t plane, float2* X, int64_t ld, hipStream_t s);
hipError_t launch_digitize(const float* wave, const float* noise, int64_t n, float gain, float baseline,
                           int bits, uint16_t* out, hipStream_t s);
// Adjoint wire pass over `batch` items sharing R (item b at Gt + b*strideG,
// S + b*strideS): grid-gradient spectra written over S; dR = (or +=, with
// accumulate) the gradient summed over the items.  The items are split in
// up to kAdjointGroups groups of blocks, as many as whole response-gradient
// partials fit in `scratch` (scratch_bytes; may be NULL: one group).
constexpr int kAdjointGroups = 4;
int wire_adjoint_groups(int batch, size_t scratch_bytes, int n_imp, int nw_fft, int nt_fft);
hipError_t launch_wire_adjoint_items(const float2* Gt, int64_t ldG, int64_t strideG, float2* S, int64_t ldS,
                                     int64_t strideS, int batch, int n_wires, int n_imp, int nw_fft,
                                     int nt_fft, const float2* R, float2* dR, float resp_scale,
                                     hipStream_t s, bool accumulate, void* scratch = nullptr,
                                     size_t scratch_bytes = 0);
hipError_t launch_sample_counts(int mode, int64_t n, const float* q, const double* p,
                                const uint32_t* ctr3, uint32_t plane, uint64_t seed, float* out,
                                hipStream_t s);

}  // namespace lar
