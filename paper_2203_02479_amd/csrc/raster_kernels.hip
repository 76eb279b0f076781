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
// Fluctuation (paper Sec. 3.1): per bin, Binomial(rint|q|, p), Poisson(|q| p)
// or the normal approximation of the binomial, with p = wt*wx, uniforms from Philox4x32-10 (Salmon et al.,
// SC'11) keyed by seed and counter (depo, event, bin, plane*2^24 + draw).
// Binomial: inversion for n*min(p,1-p) < 10, BTRD otherwise (Hormann 1993);
// Poisson: inversion for lambda < 10, PTRS otherwise (Hormann 1993).  The
// sampler is FP64 without contraction so that a CPU implementation of the
// same steps makes the same decisions.
#include <algorithm>

#include "lar_internal.hpp"

namespace lar {

// Float add to the grid in global memory.  The grid pointer arrives in a
// struct (a generic pointer), so the address space is stated here: a global
// atomic instead of a flat one.
typedef __attribute__((address_space(1))) float global_float;
__device__ __forceinline__ void grid_add(float* p, float v) {
    __hip_atomic_fetch_add((global_float*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- Philox

struct PhiloxStream {
    uint32_t k0, k1;
    uint32_t c0, c1, c2, c3;
    uint32_t b0, b1, b2, b3;
    int left;   // 0: no buffered uniform, 2: second uniform of the block left, 3: primed block
};

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
    if (s.left == 3) {
        s.left = 2;
        return u52(s.b0, s.b1);
    }
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

// Compute the stream's first Philox block now (so that lanes about to take
// different sampler branches run it together); draws are unchanged.
__device__ __forceinline__ void stream_prime(PhiloxStream& s) {
    uint32_t o0 = s.c0, o1 = s.c1, o2 = s.c2, o3 = s.c3;
    philox4x32_10(o0, o1, o2, o3, s.k0, s.k1);
    s.c3 += 1u;
    s.b0 = o0;
    s.b1 = o1;
    s.b2 = o2;
    s.b3 = o3;
    s.left = 3;   // marks a primed block: both uniforms still unread
}

// ---------------------------------------------------------------- samplers

#define LAR_MAX_TRIES 1000

// Mean (n min(p, 1-p), lambda) below which a count is drawn by inversion,
// else by the rejection samplers.
static constexpr double kInvMean = 10.0;
// Entries of the 1/k table of binom_inversion: k <= 111 is reached (the
// search stops past 110) and the next entry is loaded one step ahead.
static constexpr int kRcpTable = 113;

// log k! - [(k + 1/2) log(k+1) - (k+1) + log(2 pi)/2]
__device__ double stirling_tail(double k) {
#pragma clang fp contract(off)
    if (k < 10.0)
        return lgamma(k + 1.0) - (k + 0.5) * log(k + 1.0) + (k + 1.0) - 0.91893853320467274178;
    double r = 1.0 / (k + 1.0);
    double r2 = r * r;
    return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * r2) * r2) * r;
}

// x^n for a non-negative integer n (held in a double): square-and-multiply
// over the bits of n from the least significant, IEEE multiplies only.  When
// every active lane has the same n (the lanes of one depo) the bit loop runs
// on scalar registers; the multiplies, and so the result, are the same.
__device__ __forceinline__ double ipow_n(double x, double n) {
#pragma clang fp contract(off)
    uint64_t e = (uint64_t)n;
    double r = 1.0, b = x;
    const uint32_t lo0 = __builtin_amdgcn_readfirstlane((uint32_t)e);
    const uint32_t hi0 = __builtin_amdgcn_readfirstlane((uint32_t)(e >> 32));
    const uint64_t e0 = ((uint64_t)hi0 << 32) | lo0;
    if (__ballot(e != e0) == 0) {
        if (hi0 == 0u) {   // 32-bit exponent: the loop ends at its last bit
            uint32_t es = lo0;
            if (es) {
                for (;;) {
                    if (es & 1u) r = r * b;
                    es >>= 1;
                    if (!es) break;
                    b = b * b;
                }
            }
            return r;
        }
        for (uint64_t es = e0; es; ) {
            if (es & 1u) r = r * b;
            es >>= 1;
            if (es) b = b * b;
        }
        return r;
    }
    while (e) {
        if (e & 1u) r = r * b;
        e >>= 1;
        if (e) b = b * b;
    }
    return r;
}

// Binomial by inversion from k = 0 (p <= 1/2, n p < 10): f(0) = (1-p)^n,
// f(k) = f(k-1) ((n+1) r (1/k) - r), r = p/(1-p), 1/k correctly rounded.  When n p < 1 the first
// uniform is compared with a lower bound of f(0) first: (1-p)^n >= 1 - n p
// (Bernoulli), minus a margin above the rounding of q and of the powering,
// so the early return of 0 happens only where the full test returns 0.
// ONE_TRY: return -1 instead of redrawing when the search runs off its end
// (k = n or k > 110 reached with u left over): the stream is then not needed
// past the first uniform, which keeps the hot kernel's registers down; the
// caller redraws the bin with the full sampler.
template <bool ONE_TRY = false>
__device__ __forceinline__ double binom_inversion(double n, double p, PhiloxStream& s,
                                                  const double* rtab) {
#pragma clang fp contract(off)
    double q = 1.0 - p;
    double ratio = p / q;
    double g = ratio * (n + 1.0);
    double u = next_uniform(s);
    double np = n * p;
    if (np < 1.0 && u < (1.0 - np) - (n + 64.0) * 8.8817841970012523e-16) return 0.0;
    double f0 = ipow_n(q, n);
    for (int tries = 0; tries < (ONE_TRY ? 1 : LAR_MAX_TRIES); ++tries) {
        if (tries > 0) u = next_uniform(s);
        double f = f0;
        // the search stops past k = n or k = 110 (n is a whole number): an
        // integer bound, and an integer step counter
        const int kmax = n < 111.0 ? (int)n : 111;
        int k = 0;
        if (rtab) {
            // 1/k correctly rounded, from the table (kRcpTable entries); the
            // next step's entry is loaded one step ahead
            // one exit test per step (two exits cost the wave a set of
            // exec-mask updates per step)
            double ik_next = rtab[1];
            bool hit = u < f;
            while (!hit && k < kmax) {
                u = u - f;
                ++k;
                const double ik = ik_next;
                ik_next = rtab[k + 1];
                f = f * (g * ik - ratio);
                hit = u < f;
            }
            if (hit) return (double)k;
        } else {
            bool hit = u < f;
            while (!hit && k < kmax) {
                u = u - f;
                ++k;
                f = f * (g * (1.0 / (double)k) - ratio);
                hit = u < f;
            }
            if (hit) return (double)k;
        }
    }
    return ONE_TRY ? -1.0 : floor(n * p);
}

// BTRD's explicit test v <= f(k)/f(m) for |k - m| <= 15, with the pmf ratio
// prod (nr/i - r) written as the product of the numerators (nr - r i) over
// the product of the i's (no division).
__device__ __forceinline__ int btrd_ratio_accept(double v, double k, double m, double nr, double r) {
#pragma clang fp contract(off)
    // one loop over i in (min(k, m), max(k, m)], ascending, for either
    // order of k and m (the same products as two separate loops, without
    // running both when a wave holds lanes of each case)
    const bool up = m < k;
    const double lo = (up ? m : k) + 1.0;
    const int steps = (int)fabs(k - m);
    double num = 1.0, den = 1.0;
    for (int t = 0; t < steps; ++t) {
        const double i = lo + (double)t;
        num = num * (nr - r * i);
        den = den * i;
    }
    if (up) return v * den <= num;
    if (m > k) return v * num <= den;
    return v <= 1.0;
}

// Binomial by BTRD, transformed rejection with decomposition (p <= 1/2, n p >= 10).
// from: the first try to run, with the stream at Philox block `from` (every
// earlier try went past its immediate acceptance and took one block).
// to < LAR_MAX_TRIES: run tries [from, to) only and return -1 if none of
// them accepts (the draw then continues at try `to`).
__device__ double binom_btrd(double n, double p, PhiloxStream& s, int from = 0,
                             int to = LAR_MAX_TRIES) {
#pragma clang fp contract(off)
    // constants of the fast acceptance region first; those of the slow
    // path are formed only when it is reached (identical values)
    double npq = n * p * (1.0 - p);
    double spq = sqrt(npq);
    double b = 1.15 + 2.53 * spq;
    double a = -0.0873 + 0.0248 * b + 0.01 * p;
    double c = n * p + 0.5;
    double vr = 0.92 - 4.2 / b;
    double urvr = 0.86 * vr;
    double m = 0.0, r = 0.0, nr = 0.0, alpha = 0.0;
    bool slow_ready = false;
    for (int tries = from; tries < to; ++tries) {
        double v = next_uniform(s);
        double u;
        if (v <= urvr) {
            u = v / vr - 0.43;
            return floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
        }
        if (!slow_ready) {
            m = floor((n + 1.0) * p);
            r = p / (1.0 - p);
            nr = (n + 1.0) * r;
            alpha = (2.83 + 5.1 / b) * spq;
            slow_ready = true;
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
            if (btrd_ratio_accept(v, k, m, nr, r)) return k;
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
    if (to < LAR_MAX_TRIES) return -1.0;
    if (!slow_ready) m = floor((n + 1.0) * p);
    return m;
}

// Poisson by inversion (0 < lam < 10).  For lam < 1 the first uniform is
// compared with exp(-lam) >= 1 - lam (minus a margin above exp's rounding)
// first, which decides k = 0 exactly where the full test does.
// ONE_TRY as for binom_inversion.
template <bool ONE_TRY = false>
__device__ double poisson_inversion(double lam, PhiloxStream& s) {
#pragma clang fp contract(off)
    double u = next_uniform(s);
    if (lam < 1.0 && u < (1.0 - lam) - 1e-13) return 0.0;
    double p0 = exp(-lam);
    for (int tries = 0; tries < (ONE_TRY ? 1 : LAR_MAX_TRIES); ++tries) {
        if (tries > 0) u = next_uniform(s);
        double p = p0, cdf = p0, k = 0.0;
        while (u > cdf && !(k > 200.0)) {   // one exit test per step
            k = k + 1.0;
            p = p * lam / k;
            cdf = cdf + p;
        }
        if (u <= cdf) return k;
    }
    return ONE_TRY ? -1.0 : floor(lam);
}

// Poisson by PTRS, transformed rejection with squeeze (lam >= 10).
__device__ double poisson_ptrs(double lam, PhiloxStream& s, int from = 0,   // from, to as for binom_btrd
                               int to = LAR_MAX_TRIES) {
#pragma clang fp contract(off)
    double slam = sqrt(lam);
    double loglam = log(lam);
    double b = 0.931 + 2.53 * slam;
    double a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int tries = from; tries < to; ++tries) {
        double u = next_uniform(s) - 0.5;
        double v = next_uniform(s);
        double us = 0.5 - fabs(u);
        double k = floor((2.0 * a / us + b) * u + lam + 0.43);
        if (us >= 0.07 && v <= vr) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        if (log(v) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0))
            return k;
    }
    return to < LAR_MAX_TRIES ? -1.0 : floor(lam);
}

// BTRD without its logarithmic acceptance test: the same tries, the same
// uniforms and the same decisions as binom_btrd for as long as every try is
// decided by the fast region, the bounds test or the explicit pmf ratio
// (|k - m| <= 15); returns -1 as soon as a try needs the log-scale test, or
// after kFastTries tries.  The full sampler then redraws the bin from its
// counter and reaches the same result.  TRIES limits the tries: with
// kTryAccept only the first try's immediate-acceptance region is taken (-1
// otherwise), with 1 the whole first try: cheap stages that most bins finish
// in, run apart so that a wave's lanes stay converged.  Returns -1 - t when
// try t needs the log-scale test, kTriesUsed when every try up to TRIES was
// rejected.
//
// A try that is not accepted at once takes exactly two uniforms, one Philox
// block, so try t >= 1 starts at block t when every earlier try went past
// its immediate acceptance: binom_btrd_fast_from resumes the sampler there.
static constexpr int kFastTries = 4;
static constexpr int kTryAccept = 0;
static constexpr double kTriesUsed = -100.0;

template <int TRIES>
__device__ __forceinline__ double binom_btrd_fast(double n, double p, PhiloxStream& s, int from = 0) {
#pragma clang fp contract(off)
    double npq = n * p * (1.0 - p);
    double spq = sqrt(npq);
    double b = 1.15 + 2.53 * spq;
    double a = -0.0873 + 0.0248 * b + 0.01 * p;
    double c = n * p + 0.5;
    double vr = 0.92 - 4.2 / b;
    double urvr = 0.86 * vr;
    double m = 0.0, r = 0.0, nr = 0.0, alpha = 0.0;
    bool slow_ready = false;
    for (int tries = from; tries < (TRIES == kTryAccept ? 1 : TRIES); ++tries) {
        double v = next_uniform(s);
        double u;
        if (v <= urvr) {
            u = v / vr - 0.43;
            return floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
        }
        if (TRIES == kTryAccept) return -1.0;
        if (!slow_ready) {
            m = floor((n + 1.0) * p);
            r = p / (1.0 - p);
            nr = (n + 1.0) * r;
            alpha = (2.83 + 5.1 / b) * spq;
            slow_ready = true;
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
        if (km > 15.0) return -1.0 - tries;
        if (btrd_ratio_accept(v, k, m, nr, r)) return k;
    }
    return kTriesUsed;
}

// PTRS without its logarithmic acceptance test (same tries and decisions as
// poisson_ptrs while each try is decided by the immediate acceptance or the
// cheap rejection); -1 when a try needs the log test or after kFastTries.
// TRIES, from and the return codes as for binom_btrd_fast (every PTRS try
// takes one Philox block).
template <int TRIES>
__device__ __forceinline__ double poisson_ptrs_fast(double lam, PhiloxStream& s, int from = 0) {
#pragma clang fp contract(off)
    double slam = sqrt(lam);
    double b = 0.931 + 2.53 * slam;
    double a = -0.059 + 0.02483 * b;
    double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int tries = from; tries < (TRIES == kTryAccept ? 1 : TRIES); ++tries) {
        double u = next_uniform(s) - 0.5;
        double v = next_uniform(s);
        double us = 0.5 - fabs(u);
        double k = floor((2.0 * a / us + b) * u + lam + 0.43);
        if (us >= 0.07 && v <= vr) return k;
        if (TRIES == kTryAccept) return -1.0;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        return -1.0 - tries;
    }
    return kTriesUsed;
}

// The opening test of the inversion samplers for a small mean (n p < 1,
// lam < 1): 0 when the first uniform lies below the lower bound of the
// probability of 0 (the same test, on the same uniform, as in
// binom_inversion / poisson_inversion), -1 when the full search is needed.
__device__ __forceinline__ double binom_zero_test(double n, double p, PhiloxStream& s) {
#pragma clang fp contract(off)
    double u = next_uniform(s);
    double np = n * p;
    if (np < 1.0 && u < (1.0 - np) - (n + 64.0) * 8.8817841970012523e-16) return 0.0;
    return -1.0;
}

__device__ __forceinline__ double poisson_zero_test(double lam, PhiloxStream& s) {
#pragma clang fp contract(off)
    double u = next_uniform(s);
    if (lam < 1.0 && u < (1.0 - lam) - 1e-13) return 0.0;
    return -1.0;
}

// Signed count of one bin drawn with inversion or the rejection samplers'
// fast region only; returns NaN when the bin needs the full rejection
// sampler (bin_count_in<true>, which redraws it from the same counter).
// Stages (a bin of a given regime may be drawn by the cheap stage first and,
// when that returns NaN, by the full one from the same counter, with the
// same result as the full stage alone):
//   kStageZero  small-mean bins: the zero test only
//   kStageInv   every non-rejection bin: the full inversion
//   kStageFirst  rejection bins: the first try's immediate acceptance only
//   kStageSecond rejection bins: the whole first try
//   kStageRej    rejection bins: the fast rejection sampler
//   kStageResume rejection bins whose first try went past its immediate
//                acceptance and was rejected: the fast rejection sampler
//                from the second try (stream at block 1)
//   kStageAll    any bin: inversion or the fast rejection sampler by regime
// Undecided bins return NaN.  For the rejection stages, *next (when given)
// then holds where the draw continues: the try t that needs the log-scale
// test (encoded t), or, when every try of the stage was rejected, the next
// try for the fast sampler (encoded kNextFast + t).
enum { kStageZero = 0, kStageInv = 1, kStageFirst = 2, kStageRej = 3, kStageAll = 4, kStageSecond = 5,
       kStageResume = 6 };
static constexpr int kNextFast = 16;

__device__ __forceinline__ int next_try(double code, int tries_of_stage) {
    return code == kTriesUsed ? kNextFast + tries_of_stage : (int)(-1.0 - code);
}

// VALID: the caller guarantees n > 0 (lam > 0) and 0 < p < 1 (the bins of
// k_raster's inversion and rejection stacks), so the trivial cases are not
// tested.
template <int MODE, int STAGE, bool VALID = false>
__device__ __forceinline__ float bin_count_fast(float q, double p, uint64_t seed, uint32_t depo,
                                                uint32_t event, uint32_t bin, uint32_t plane,
                                                const double* rtab = nullptr, int* next = nullptr) {
#pragma clang fp contract(off)
    PhiloxStream s;
    stream_init(s, seed, depo, event, bin, plane);
    if (STAGE == kStageResume)
        s.c3 += 1u;          // the second try's block
    else
        stream_prime(s);
    const int from = STAGE == kStageResume ? 1 : 0;
    double aq = fabs((double)q);
    double r;
    if (MODE == 1) {
        double n = rint(aq);
        if (!VALID && (!(n > 0.0) || !(p > 0.0))) {
            r = 0.0;
        } else if (!VALID && p >= 1.0) {
            r = n;
        } else {
            bool flip = p > 0.5;
            double pp = flip ? 1.0 - p : p;
            double k;
            if (STAGE == kStageResume)
                k = binom_btrd_fast<kFastTries>(n, pp, s, from);
            else if (STAGE == kStageZero)
                k = binom_zero_test(n, pp, s);
            else if (STAGE == kStageFirst)
                k = binom_btrd_fast<kTryAccept>(n, pp, s);
            else if (STAGE == kStageSecond)
                k = binom_btrd_fast<1>(n, pp, s);
            else if (STAGE == kStageRej)
                k = binom_btrd_fast<kFastTries>(n, pp, s);
            else if (STAGE == kStageInv)
                k = binom_inversion<true>(n, pp, s, rtab);
            else
                k = (n * pp < kInvMean) ? binom_inversion(n, pp, s, rtab) : binom_btrd_fast<kFastTries>(n, pp, s);
            if (k < 0.0) {
                if (next) *next = next_try(k, STAGE == kStageSecond ? 1 : kFastTries);
                return __builtin_nanf("");
            }
            r = flip ? n - k : k;
        }
    } else {
        double lam = aq * p;
        if (!VALID && !(lam > 0.0)) {
            r = 0.0;
        } else {
            if (STAGE == kStageResume)
                r = poisson_ptrs_fast<kFastTries>(lam, s, from);
            else if (STAGE == kStageZero)
                r = poisson_zero_test(lam, s);
            else if (STAGE == kStageFirst)
                r = poisson_ptrs_fast<kTryAccept>(lam, s);
            else if (STAGE == kStageSecond)
                r = poisson_ptrs_fast<1>(lam, s);
            else if (STAGE == kStageRej)
                r = poisson_ptrs_fast<kFastTries>(lam, s);
            else if (STAGE == kStageInv)
                r = poisson_inversion<true>(lam, s);
            else
                r = (lam < kInvMean) ? poisson_inversion(lam, s) : poisson_ptrs_fast<kFastTries>(lam, s);
            if (r < 0.0) {
                if (next) *next = next_try(r, STAGE == kStageSecond ? 1 : kFastTries);
                return __builtin_nanf("");
            }
        }
    }
    float f = (float)r;
    return q < 0.f ? -f : f;
}

// Whether a bin's draw takes the rejection samplers (BTRD / PTRS) rather
// than inversion or a trivial case: mode 1 with n min(p,1-p) >= 10, mode 2
// with lambda >= 10.
__device__ __forceinline__ bool rejection_regime(int mode, float q, double p) {
#pragma clang fp contract(off)
    double aq = fabs((double)q);
    if (mode == 1) {
        double n = rint(aq);
        if (!(n > 0.0) || !(p > 0.0) || p >= 1.0) return false;
        double pp = p > 0.5 ? 1.0 - p : p;
        return !(n * pp < kInvMean);
    }
    double lam = aq * p;
    return lam > 0.0 && !(lam < kInvMean);
}

// Wave-local stacks of k_raster, by the first sampler stage of a bin:
//   kStkZ  small mean (mode 1: n min(p,1-p) < 1; mode 2: lam < 1) and bins
//          without randomness (n = 0, p = 0, p >= 1): kStageZero
//   kStkI  mean in [1, 4): kStageInv       kStkJ  mean in [4, 10): kStageInv
//   kStkF  the rejection regime (mean >= 10): kStageFirst
// Inversion takes about mean + 1 steps; splitting its bins at a mean of 4
// keeps the steps of the lanes of one batch close together.  The numbering
// is k_raster's drawing priority (I, J, Z, F).
enum { kStkI = 0, kStkJ = 1, kStkZ = 2, kStkF = 3, kStacks = 4 };

// The same classification from the float product pf (p = (double)pf) in
// float arithmetic: only the rejection boundary (mean 10) must agree with
// the samplers' own FP64 test, and a float mean more than 1e-4 away from 10
// is on the same side of it (float rounding here is below 1e-6 relative);
// the few bins closer to it take the FP64 test.  The other boundaries only
// pick a stack.
__device__ __forceinline__ int sampler_stack(int mode, float q, double p);

__device__ __forceinline__ int sampler_stack_f(int mode, float q, float pf) {
    const float aq = fabsf(q);
    float mean;
    if (mode == 1) {
        const float n = rintf(aq);
        if (!(n > 0.f) || !(pf > 0.f) || pf >= 1.f) return kStkZ;
        mean = n * (pf > 0.5f ? 1.f - pf : pf);
    } else {
        mean = aq * pf;
        if (!(mean > 0.f)) return kStkZ;
    }
    if (mean > 9.999f && mean < 10.001f) return sampler_stack(mode, q, (double)pf);
    return mean >= 10.f ? kStkF : mean < 1.f ? kStkZ : mean < 4.f ? kStkI : kStkJ;
}

__device__ __forceinline__ int sampler_stack(int mode, float q, double p) {
#pragma clang fp contract(off)
    double aq = fabs((double)q);
    double mean;
    if (mode == 1) {
        double n = rint(aq);
        if (!(n > 0.0) || !(p > 0.0) || p >= 1.0) return kStkZ;
        double pp = p > 0.5 ? 1.0 - p : p;
        mean = n * pp;
    } else {
        mean = aq * p;
        if (!(mean > 0.0)) return kStkZ;
    }
    return !(mean < kInvMean) ? kStkF : mean < 1.0 ? kStkZ : mean < 4.0 ? kStkI : kStkJ;
}

// Signed count of one bin, for a bin known to be in the given regime.
// from > 0 (rejection regime only): resume at try `from`, every earlier try
// having gone past its immediate acceptance (one Philox block each).
// to (rejection regime): stop after try to - 1, NaN if no try accepted.
template <bool REJECT>
__device__ __forceinline__ float bin_count_in(int mode, float q, double p, uint64_t seed,
                                              uint32_t depo, uint32_t event, uint32_t bin,
                                              uint32_t plane, int from = 0, int to = LAR_MAX_TRIES) {
#pragma clang fp contract(off)
    PhiloxStream s;
    stream_init(s, seed, depo, event, bin, plane);
    s.c3 += (uint32_t)from;
    double aq = fabs((double)q);
    double r;
    if (mode == 1) {
        double n = rint(aq);
        if (!(n > 0.0) || !(p > 0.0)) {
            r = 0.0;
        } else if (p >= 1.0) {
            r = n;
        } else {
            bool flip = p > 0.5;
            double pp = flip ? 1.0 - p : p;
            double k = REJECT ? binom_btrd(n, pp, s, from, to) : binom_inversion(n, pp, s, nullptr);
            if (k < 0.0) return __builtin_nanf("");
            r = flip ? n - k : k;
        }
    } else {
        double lam = aq * p;
        r = !(lam > 0.0) ? 0.0 : (REJECT ? poisson_ptrs(lam, s, from, to) : poisson_inversion(lam, s));
        if (r < 0.0) return __builtin_nanf("");
    }
    float f = (float)r;
    return q < 0.f ? -f : f;
}

// Signed count of one bin under the normal approximation of
// Binomial(n = rint|q|, p) (mode 3; paper Sec. 3.1: the GPU port's choice):
// mu = n p, sd = sqrt(mu (1 - p)), count = rint(mu + sd z) clipped to [0, n],
// with z = sqrt(-2 log u1) cos(2 pi u2) (Box and Muller 1958) on the two
// uniforms of the bin's first Philox block.  One block per bin, no branch
// on the draw.
__device__ __forceinline__ float bin_count_normal(float q, double p, uint64_t seed, uint32_t depo,
                                                  uint32_t event, uint32_t bin, uint32_t plane) {
#pragma clang fp contract(off)
    const double n = rint(fabs((double)q));
    double r;
    if (!(n > 0.0) || !(p > 0.0)) {
        r = 0.0;
    } else if (p >= 1.0) {
        r = n;
    } else {
        uint32_t c0 = depo, c1 = event, c2 = bin, c3 = plane << 24;
        philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u1 = u52(c0, c1), u2 = u52(c2, c3);
        const double rad = sqrt(-2.0 * log(u1));
        const double z = rad * cos(6.283185307179586 * u2);
        const double mu = n * p;
        const double sd = sqrt(mu * (1.0 - p));
        r = rint(mu + sd * z);
        r = r < 0.0 ? 0.0 : (r > n ? n : r);
    }
    const float f = (float)r;
    return q < 0.f ? -f : f;
}

// Signed count of one bin: sign(q) * Binomial(rint|q|, p) or Poisson(|q| p),
// or the normal approximation of the binomial (mode 3).
__device__ __forceinline__ float bin_count(int mode, float q, double p, uint64_t seed, uint32_t depo,
                                           uint32_t event, uint32_t bin, uint32_t plane) {
    if (mode == 3) return bin_count_normal(q, p, seed, depo, event, bin, plane);
    return rejection_regime(mode, q, p)
               ? bin_count_in<true>(mode, q, p, seed, depo, event, bin, plane)
               : bin_count_in<false>(mode, q, p, seed, depo, event, bin, plane);
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
#pragma clang fp contract(off)
    return 0.5f * erfcf(fabsf(z) * 0.70710678118654752f);
}

// Edge e's standardized coordinate (FP64 subtraction, then FP32).
__device__ __forceinline__ float edge_z(double org, double wd, int e, double mu, double inv_sg) {
#pragma clang fp contract(off)
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
//
// Every wave works alone on sub-chunks of kSub consecutive depos: windows,
// weights into its LDS slots, patches summed into its private LDS tile over
// the sub-chunk's bounding box, then one global float atomic per non-zero
// tile cell.  The mean path covers one depo per instruction, so no two
// lanes of an instruction share a tile cell and the tile takes plain LDS
// read-add-write; the fluctuated path draws batches that mix depos and adds
// with LDS float atomics.  Sub-chunks whose box exceeds the tile go straight
// to global atomics.
//
// Fluctuation runs in several kernels so that the hot one stays small in
// registers: k_raster draws every bin by inversion or in the rejection
// samplers' fast region and queues the rest in the workspace;
// k_raster_deferred and k_raster_hard redraw the queued bins with the rest
// of the samplers; k_raster_flagged takes the sub-chunks whose queue
// reservation did not fit and the depos too wide for the weight slots.  A
// bin's count depends only on its counter, so which kernel draws it does
// not change the result.

static constexpr int kRasterThreads = 256;
static constexpr int kWaves = kRasterThreads / 64;
static constexpr int kSub = kRasterSub;   // depos per wave sub-chunk
static constexpr int kMaxT = 16;          // window limits of the LDS slots (bins)
static constexpr int kMaxX = 32;
static constexpr int kSlot = kMaxT + kMaxX + 1;
static constexpr int kWaveQueue = 256;    // deferred bins buffered per wave
// k_raster's grid is capped at this many workgroups per CU; below the cap
// every wave takes one sub-chunk and the workgroup dispatcher balances the
// uneven sub-chunks (a persistent grid of 8 per CU, about 4 sub-chunks per
// wave, was 13% slower on track depos)
static constexpr int kRasterGroupsPerCU = 64;
static constexpr int kDeferredGroupsPerCU = 8;   // a multiple of the queue's parts
static constexpr uint32_t kInvalid = 0xFFFFFFFFu;

// Deferred bin: item, depo index within the item, bin index m * n_ticks + j
// (the bin's counter word), bin probability (float).
struct DeferredBin {
    uint32_t item, depo, bin;
    float p;
};
static_assert(sizeof(DeferredBin) == kDeferredBytes, "queue record size");

// Workspace of a fluctuated raster: header, one flag byte per sub-chunk,
// then the queue.  The queue capacity is whatever the workspace holds.
// The queue is split in kQueueParts equal parts, each with its own counter
// (k_raster's workgroup b reserves in part b mod kQueueParts): the
// reservations, one per wave, spread over several addresses instead of
// serialising on one.
static constexpr int kQueueParts = 8;
struct QueueCounter {
    unsigned long long v;        // bins queued in the part (may exceed its room)
    unsigned long long pad[3];   // one counter per 32 bytes
};
struct RasterWs {
    QueueCounter count[kQueueParts];
};
static_assert(sizeof(RasterWs) <= 256, "raster workspace header");
static_assert(kDeferredGroupsPerCU % kQueueParts == 0, "queue kernels take one part per workgroup");

// Workgroup b of k_raster_deferred and k_raster_hard works on part
// b mod kQueueParts (their grids are multiples of kQueueParts): the entries
// of one sub-chunk, and so its overflow flag, belong to one part.
static constexpr uint32_t kHardMark = 0x80000000u;   // DeferredBin::item bit: left to k_raster_hard
static constexpr uint32_t kInvMark = 0x08000000u;    // ... an inversion bin (else a rejection one)
// sub-chunk flag bits (one byte per sub-chunk, cleared by k_raster_reset)
static constexpr int kFlagOverflow = 1;   // some of its deferred bins did not fit in the queue
static constexpr int kFlagWide = 2;       // it holds a depo wider than the weight slots

size_t raster_ws_fixed_subs(int64_t nsub) { return 256 + (((size_t)nsub + 255) / 256) * 256; }

size_t raster_ws_fixed(int64_t n) { return raster_ws_fixed_subs(raster_subchunks(n)); }

// The item owning global sub-chunk g: the one given by value when there is
// no table, else a binary search over the items' first sub-chunks.
__device__ __forceinline__ int item_of(const RasterItem* items, int n_items, int64_t g) {
    if (!items) return 0;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (items[mid].sub_begin <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool depo_finite(float a, float b, float c, float d, float e) {
    return isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d) && isfinite(e);
}

// Min / max over the first kSub lanes (the only ones holding values), as a
// scalar loop over lane reads: no LDS round trips (a shuffle reduction is a
// chain of ds_bpermute).
__device__ __forceinline__ int sub_min(int v) {
    int r = __builtin_amdgcn_readlane(v, 0);
#pragma unroll
    for (int l = 1; l < kSub; ++l) r = min(r, __builtin_amdgcn_readlane(v, l));
    return r;
}
__device__ __forceinline__ int sub_max(int v) {
    int r = __builtin_amdgcn_readlane(v, 0);
#pragma unroll
    for (int l = 1; l < kSub; ++l) r = max(r, __builtin_amdgcn_readlane(v, l));
    return r;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Writes a wave's nq buffered deferred bins (codes in sq) to its queue part
// at reservation gb (room capr per part).  A reservation that does not fit
// writes invalid records in the room it has and returns false: the
// sub-chunk is then flagged for k_raster_flagged.
__device__ __forceinline__ bool queue_write(DeferredBin* queue, int part, unsigned long long capr,
                                            unsigned long long gb, int nq, const uint16_t* sq,
                                            const float* W, const int* mlo_, const int* jlo_, uint32_t item,
                                            int64_t base, uint32_t nticks, int lane) {
    const bool fits = gb + (unsigned long long)nq <= capr;
    for (int e = lane; e < nq; e += 64) {
        if (gb + (unsigned long long)e >= capr) continue;
        const unsigned long long slot = (unsigned long long)part * capr + gb + e;
        DeferredBin db;
        db.item = item;
        if (fits) {
            const int cd = sq[e];
            const int dq = (cd >> 9) & 15, a = (cd >> 4) & 31, b = cd & 15;
            if (cd & 8192) db.item |= kHardMark | kInvMark;
            const float* w = W + dq * kSlot;
            db.depo = (uint32_t)(base + dq);
            db.bin = (uint32_t)(mlo_[dq] + a) * nticks + (uint32_t)(jlo_[dq] + b);
            db.p = w[b] * w[kMaxT + a];
        } else {
            db.depo = kInvalid; db.bin = 0; db.p = 0.f;
        }
        queue[slot] = db;
    }
    return fits;
}

// 5 waves per SIMD: the sampler stages fit 96 VGPRs, and the LDS of a
// workgroup (about 29 KB with a 512-float tile) lets 5 workgroups share a
// CU; with a 768-float tile (about 33 KB) 4 do
template <int MODE, int TILE>
__global__ __launch_bounds__(kRasterThreads) __attribute__((amdgpu_waves_per_eu(TILE > 640 ? 4 : 5, 8)))
void k_raster(RasterItem one, const RasterItem* __restrict__ items, int n_items, int64_t total_sub,
              RasterWs* __restrict__ ws, uint8_t* __restrict__ flags, DeferredBin* __restrict__ queue,
              unsigned long long cap) {
    constexpr bool FLUCT = MODE != 0;
    __shared__ float s_w[kWaves][kSub * kSlot];
    __shared__ float s_tile[kWaves][TILE];
    __shared__ int s_meta[kWaves][4][kSub];            // jlo, nt, mlo, nx (nt<0 / nx<0: point axis)
    __shared__ float s_q[kWaves][kSub];
    __shared__ int s_off[kWaves][FLUCT ? kSub + 1 : 1];
    __shared__ uint16_t s_queue[kWaves][FLUCT ? kWaveQueue : 1];   // (depo:4 | row:5 | tick:4)
    __shared__ uint16_t s_list[kWaves][kStacks][FLUCT ? 128 : 1];    // cells by sampler stack
    __shared__ double s_rcp[FLUCT ? kRcpTable : 1];                  // 1/k, k < kRcpTable

    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float* W = s_w[wv];
    float* tile = s_tile[wv];
    int* jlo_ = s_meta[wv][0];
    int* nt_ = s_meta[wv][1];
    int* mlo_ = s_meta[wv][2];
    int* nx_ = s_meta[wv][3];
    float* q_ = s_q[wv];
    for (int i = lane; i < TILE; i += 64) tile[i] = 0.f;
    if (FLUCT) {
        for (int i = threadIdx.x; i < kRcpTable; i += kRasterThreads) s_rcp[i] = i ? 1.0 / (double)i : 0.0;
        __syncthreads();
    }

    for (int64_t gsub = (int64_t)blockIdx.x * kWaves + wv; gsub < total_sub;
         gsub += (int64_t)gridDim.x * kWaves) {
        const int it = item_of(items, n_items, gsub);
        const RasterItem& I = items ? items[it] : one;
        const RasterArgs& A = I.A;
        const float* __restrict__ Q = I.q;
        const float* __restrict__ Tm = I.t;
        const float* __restrict__ X = I.x;
        const float* __restrict__ ST = I.st;
        const float* __restrict__ SX = I.sx;
        float* __restrict__ grid = I.grid;
        const int64_t n = I.n;
        const int64_t base = (gsub - I.sub_begin) * kSub;
        // ---- windows: lane d < kSub takes depo base + d
        int nt = 0, nx = 0, jlo = 0, mlo = 0, cells = 0;
        bool wide = false;
        int bj0 = INT_MAX, bj1 = INT_MIN, bm0 = INT_MAX, bm1 = INT_MIN;
        if (lane < kSub) {
            int64_t d = base + lane;
            float q = 0.f;
            if (d < n) {
                q = Q[d];
                float t = Tm[d], x = X[d], st = ST[d], sx = SX[d];
                if (depo_finite(q, t, x, st, sx)) {
                    Window wt = axis_window(t, st, A.nsig, A.org_t, A.wd_t, A.n_ticks);
                    Window wx = wt.n ? axis_window(x, sx, A.nsig, A.org_x, A.wd_x, A.n_rows)
                                     : Window{0, 0, false};
                    if (wt.n && wx.n && wt.n <= kMaxT && wx.n <= kMaxX) {
                        nt = wt.point ? -wt.n : wt.n;
                        nx = wx.point ? -wx.n : wx.n;
                        jlo = wt.lo;
                        mlo = wx.lo;
                        cells = wt.n * wx.n;
                        bj0 = jlo; bj1 = jlo + wt.n - 1; bm0 = mlo; bm1 = mlo + wx.n - 1;
                    } else {
                        wide = wt.n && wx.n;
                    }
                }
            }
            jlo_[lane] = jlo; nt_[lane] = nt; mlo_[lane] = mlo; nx_[lane] = nx; q_[lane] = q;
        }
        // wave-uniform bounds, held in scalar registers
        const int jmin = sub_min(bj0), jmax = sub_max(bj1);
        const int mmin = sub_min(bm0), mmax = sub_max(bm1);
        // wave-uniform flag byte of this sub-chunk, stored at its end
        int fl = (FLUCT && __ballot(wide)) ? kFlagWide : 0;
        if (jmax < jmin) {   // no regular depo in this sub-chunk (uniform)
            if (fl && lane == 0) flags[gsub] = (uint8_t)fl;
            continue;
        }
        const int span_t = jmax - jmin + 1, span_x = mmax - mmin + 1;
        const bool use_tile = span_t * span_x <= TILE;
        if (FLUCT) {   // exclusive prefix of cell counts over the sub-chunk (scalar)
            int acc = 0, mine = 0;
#pragma unroll
            for (int l = 0; l < kSub; ++l) {
                if (lane == l) mine = acc;
                acc += __builtin_amdgcn_readlane(cells, l);
            }
            if (lane < kSub) s_off[wv][lane] = mine;
            if (lane == kSub) s_off[wv][kSub] = acc;
        }
        // ---- weights: lanes 0..kSub-1 time axis, kSub..2kSub-1 pitch axis
        {
            const int d = lane & (kSub - 1);
            const int64_t gd = base + d;
            const int ntd = __shfl(nt, d, 64), nxd = __shfl(nx, d, 64);
            const int jlod = __shfl(jlo, d, 64), mlod = __shfl(mlo, d, 64);
            if (lane < 2 * kSub && ntd != 0) {
                float* w = W + d * kSlot;
                if (lane < kSub) {
                    Window win{jlod, abs(ntd), ntd < 0};
                    axis_weights(Tm[gd], ST[gd], A.org_t, A.wd_t, win, w, 1);
                } else {
                    Window win{mlod, abs(nxd), nxd < 0};
                    axis_weights(X[gd], SX[gd], A.org_x, A.wd_x, win, w + kMaxT, 1);
                }
            }
        }
        wave_lds_sync();

        int nq = 0;   // wave-uniform count of the wave's buffered deferred bins
        const int part = (int)(blockIdx.x % kQueueParts);
        const unsigned long long capr = cap / kQueueParts;
        if (!FLUCT) {
            // ---- mean patches: one depo per instruction, lanes = rows x TW ticks
            for (int d = 0; d < kSub; ++d) {
                const int ntd = nt_[d];
                if (ntd == 0) continue;
                const int ant = abs(ntd), anx = abs(nx_[d]);
                const int sh = ant <= 4 ? 2 : (ant <= 8 ? 3 : 4);
                const int b = lane & ((1 << sh) - 1);
                const int r0 = lane >> sh, step = 64 >> sh;
                if (b < ant) {
                    const float* w = W + d * kSlot;
                    const float qwt = q_[d] * w[b];
                    const int j = jlo_[d] + b, m0 = mlo_[d];
                    if (use_tile) {
                        float* trow = tile + (m0 - mmin) * span_t + (j - jmin);
                        for (int a = r0; a < anx; a += step) trow[a * span_t] += qwt * w[kMaxT + a];
                    } else {
                        for (int a = r0; a < anx; a += step)
                            grid_add(&grid[(int64_t)(m0 + a) * A.ld + j], qwt * w[kMaxT + a]);
                    }
                }
                // other lanes touch these cells for the next depo: keep program order
                asm volatile("" ::: "memory");
            }
        } else if constexpr (MODE == 3) {
            // ---- normal-approximation patches: every cell takes one Philox
            // block and no data-dependent stage, so the cells are drawn 64 at
            // a time in order (a batch mixes depos: LDS atomics on the tile)
            const int total = __builtin_amdgcn_readfirstlane(s_off[wv][kSub]);
            const uint64_t seed = A.seed;
            const uint32_t event = A.event, plane = A.plane, nticks = (uint32_t)A.n_ticks;
            const int64_t ld = A.ld;
            int d = 0;
            for (int c0 = 0; c0 < total; c0 += 64) {
                const int c = c0 + lane;
                if (c < total) {
                    while (s_off[wv][d + 1] <= c) ++d;
                    const int ant = abs(nt_[d]);
                    const int local = c - s_off[wv][d];
                    const int a = (int)(((float)local + 0.5f) * (1.0f / (float)ant));
                    const int b = local - a * ant;
                    const float* w = W + d * kSlot;
                    const int j = jlo_[d] + b, m = mlo_[d] + a;
                    const double p = (double)(w[b] * w[kMaxT + a]);
                    const float v = bin_count_normal(q_[d], p, seed, (uint32_t)(base + d), event,
                                                     (uint32_t)m * nticks + (uint32_t)j, plane);
                    if (v != 0.f) {
                        if (use_tile)
                            atomicAdd(&tile[(m - mmin) * span_t + (j - jmin)], v);
                        else
                            grid_add(&grid[(int64_t)m * ld + j], v);
                    }
                }
            }
        } else {
            // ---- fluctuated patches.  Cells are classified 64 at a time by
            // sampler stage into four wave-local stacks, and each stack is
            // drawn in batches of 64 so that a wave runs one sampler stage at
            // a time:
            //   Z  small-mean bins (n p < 1, lam < 1) and degenerate ones:
            //      the zero test only; a bin that fails it moves to I
            //   I, J  inversion bins of mean below / above 4: the full inversion
            //   F  rejection bins: the first try's immediate acceptance; a bin
            //      that needs more is queued for k_raster_deferred, which runs
            //      the rest of the rejection sampler (its registers would
            //      otherwise bound this kernel's occupancy).
            // A moved or queued bin is redrawn from its counter, so every
            // stage reaches the count of the one-shot sampler.  Stacks hold
            // up to 128 codes.  A batch is drawn from the first stack, in the
            // order I, J, Z, F, that holds 64 codes or more (any, once every
            // cell is classified); new cells are classified only when all
            // stacks hold fewer than 64.  I comes before Z, which pushes into
            // it, so every push of up to 64 codes fits.
            const int total = __builtin_amdgcn_readfirstlane(s_off[wv][kSub]);
            uint16_t* const L0 = s_list[wv][0];   // stack k at L0 + 128 k
            // the item's constants, read once (not per batch through the
            // item-or-table reference)
            const uint64_t seed = A.seed;
            const uint32_t event = A.event, plane = A.plane, nticks = (uint32_t)A.n_ticks;
            const int64_t ld = A.ld;
            // wave-uniform stack sizes (each below 128), byte k = stack k, so
            // that the first stack holding thr or more codes is the lowest
            // set bit of a mask
            uint32_t nL = 0u;
            int d = 0;
            int c0 = 0;
            for (;;) {
                const bool tail = c0 >= total;
                // bytes >= 64: bit 6; bytes >= 1: bit 7 of byte + 127
                const uint32_t ready = tail ? ((nL + 0x7f7f7f7fu) & 0x80808080u) : (nL & 0x40404040u);
                if (ready) {   // one batch of 64 (or the rest) from stack st (wave-uniform)
                    const int st = __builtin_ctz(ready) >> 3;
                    const int nst = (int)((nL >> (8 * st)) & 0xffu);
                    wave_lds_sync();
                    const int cnt = min(nst, 64);
                    int code = 0, m = 0, j = 0;
                    bool todo = false, defer = false, move = false;
                    float v = 0.f;
                    if (lane < cnt) {
                        code = L0[st * 128 + nst - cnt + lane];
                        const int dd = code >> 9, a = (code >> 4) & 31, b = code & 15;
                        const float* w = W + dd * kSlot;
                        j = jlo_[dd] + b;
                        m = mlo_[dd] + a;
                        const double p = (double)(w[b] * w[kMaxT + a]);
                        const uint32_t bin = (uint32_t)m * nticks + (uint32_t)j;
                        const uint32_t dg = (uint32_t)(base + dd);
                        if (st == kStkZ)
                            v = bin_count_fast<MODE, kStageZero>(q_[dd], p, seed, dg, event, bin, plane);
                        else if (st == kStkF)
                            v = bin_count_fast<MODE, kStageFirst, true>(q_[dd], p, seed, dg, event, bin, plane);
                        else
                            v = bin_count_fast<MODE, kStageInv, true>(q_[dd], p, seed, dg, event, bin, plane,
                                                                s_rcp);
                        if (v != v) {   // Z: to I; I, J (search ran off its end) and F: queued
                            if (st == kStkZ) move = true;
                            else defer = true;
                        } else if (v != 0.f) {
                            todo = true;
                        }
                    }
                    nL -= (uint32_t)cnt << (8 * st);
                    const uint64_t below = (1ull << lane) - 1;
                    if (st == kStkZ) {   // failed zero tests go to the low-mean inversion stack
                        const uint64_t mm = __ballot(move);
                        const int nI = (int)((nL >> (8 * kStkI)) & 0xffu);
                        if (move) L0[kStkI * 128 + nI + __popcll(mm & below)] = (uint16_t)code;
                        nL += (uint32_t)__popcll(mm) << (8 * kStkI);
                    }
                    if (st != kStkZ) {
                        const uint64_t dm = __ballot(defer);
                        // bit 13 of a queued code: an inversion bin (full inversion in k_raster_hard)
                        if (defer)
                            s_queue[wv][nq + __popcll(dm & below)] = (uint16_t)(code | (st != kStkF ? 8192 : 0));
                        nq += __popcll(dm);
                    }
                    // add the drawn counts: two depos of one batch may share a cell,
                    // so the tile takes LDS atomics here (cheaper than serialising
                    // the lanes by depo, measured)
                    if (todo) {
                        if (use_tile)
                            atomicAdd(&tile[(m - mmin) * span_t + (j - jmin)], v);
                        else
                            grid_add(&grid[(int64_t)m * ld + j], v);
                    }
                    // move queued bins to the workspace when the next batch could
                    // overflow the buffer (the rest after the sub-chunk's tile
                    // flush, which hides the wait for the reservation)
                    if (nq > kWaveQueue - 64) {
                        wave_lds_sync();
                        unsigned long long gb = 0;
                        if (lane == 0) gb = atomicAdd(&ws->count[part].v, (unsigned long long)nq);
                        gb = __shfl(gb, 0, 64);
                        if (!queue_write(queue, part, capr, gb, nq, s_queue[wv], W, mlo_, jlo_, (uint32_t)it, base,
                                         nticks, lane))
                            fl |= kFlagOverflow;
                        nq = 0;
                        wave_lds_sync();
                    }
                    continue;
                }
                if (tail) break;
                // classify the next 64 cells (every stack holds < 64)
                const int c = c0 + lane;
                int sk = -1, code = 0;
                if (c < total) {
                    while (s_off[wv][d + 1] <= c) ++d;
                    const int ant = abs(nt_[d]);
                    const int local = c - s_off[wv][d];
                    const int a = (int)(((float)local + 0.5f) * (1.0f / (float)ant));
                    const int b = local - a * ant;
                    const float* w = W + d * kSlot;
                    code = (d << 9) | (a << 4) | b;
                    sk = sampler_stack_f(MODE, q_[d], w[b] * w[kMaxT + a]);
                }
                const uint64_t below = (1ull << lane) - 1;
#pragma unroll
                for (int k = 0; k < kStacks; ++k) {
                    const uint64_t mk = __ballot(sk == k);
                    if (sk == k) L0[k * 128 + (int)((nL >> (8 * k)) & 0xffu) + __popcll(mk & below)] = (uint16_t)code;
                    nL += (uint32_t)__popcll(mk) << (8 * k);
                }
                c0 += 64;
            }
        }
        // the last queue reservation is requested before the tile flush and
        // used after it
        unsigned long long gb = 0;
        if (FLUCT && nq > 0) {
            wave_lds_sync();
            if (lane == 0) gb = atomicAdd(&ws->count[part].v, (unsigned long long)nq);
        }
        // ---- flush: one global atomic per non-zero cell, leave the tile zeroed
        if (use_tile) {
            const int area = span_t * span_x;
            for (int e = lane; e < area; e += 64) {
                float v = tile[e];
                if (v != 0.f) {
                    int r = e / span_t, ci = e - r * span_t;
                    grid_add(&grid[(int64_t)(mmin + r) * A.ld + jmin + ci], v);
                    tile[e] = 0.f;
                }
            }
        }
        if (FLUCT && nq > 0) {
            gb = __shfl(gb, 0, 64);
            if (!queue_write(queue, part, capr, gb, nq, s_queue[wv], W, mlo_, jlo_, (uint32_t)it, base,
                             (uint32_t)A.n_ticks, lane))
                fl |= kFlagOverflow;
            wave_lds_sync();
        }
        if (FLUCT && fl && lane == 0) flags[gsub] = (uint8_t)fl;
    }
}

// Clears the queue counter and the sub-chunk flags.
__global__ void k_raster_reset(RasterWs* ws, uint8_t* flags, int64_t nsub) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kQueueParts) ws->count[i].v = 0ull;
    for (; i < nsub; i += (int64_t)gridDim.x * blockDim.x) flags[i] = 0;
}

// The queued bins (skipping those of sub-chunks left to k_raster_flagged),
// in two converged stages per wave: every bin first runs the whole first try
// of the rejection sampler; the bins whose first try was rejected resume the
// fast sampler at the second try (up to kFastTries), collected in a
// wave-local stack and drawn 64 at a time.  Bins that reach the log-scale
// test or use up the fast tries are marked for k_raster_hard.  The full
// sampler is not compiled in here, so this kernel keeps a small register
// footprint.  A bin's count depends only on its counter, so the stage that
// draws it does not change it.
static constexpr int kDefWaves = 4;

__device__ __forceinline__ void deferred_add(const RasterItem& one, const RasterItem* items,
                                             const DeferredBin& db, float v) {
    const RasterItem& I = items ? items[db.item] : one;
    const int64_t m = db.bin / (uint32_t)I.A.n_ticks, j = db.bin - m * I.A.n_ticks;
    grid_add(&I.grid[m * I.A.ld + j], v);
}

template <int MODE, int STAGE>
__device__ __forceinline__ float deferred_draw(const RasterItem& one, const RasterItem* items,
                                               const DeferredBin& db, int* next) {
    const RasterItem& I = items ? items[db.item] : one;
    const RasterArgs& A = I.A;
    return bin_count_fast<MODE, STAGE>(I.q[db.depo], (double)db.p, A.seed, db.depo, A.event, db.bin,
                                       A.plane, nullptr, next);
}

// Marks queue entry idx for k_raster_hard, which resumes the full sampler at
// try t (a plain store to the entry this lane owns: no shared counter, whose
// atomics would serialise on one address).
static constexpr uint32_t kHardTryShift = 28;   // DeferredBin::item bits 28-30: t
__device__ __forceinline__ void defer_hard(DeferredBin* queue, uint32_t idx, int t) {
    queue[idx].item |= kHardMark | ((uint32_t)t << kHardTryShift);
}

template <int MODE>
__global__ __launch_bounds__(kDefWaves * 64) __attribute__((amdgpu_waves_per_eu(5, 8)))
void k_raster_deferred(
    RasterItem one, const RasterItem* __restrict__ items, RasterWs* __restrict__ ws,
    const uint8_t* __restrict__ flags, DeferredBin* __restrict__ queue, unsigned long long cap) {
    __shared__ uint32_t s_stk[kDefWaves][128];   // queue indices of resumed bins
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* S1 = s_stk[wv];
    const unsigned part = blockIdx.x % kQueueParts;
    const unsigned long long capr = cap / kQueueParts, used = ws->count[part].v;
    const unsigned long long cnt = min(used, capr);
    DeferredBin* const pq = queue + part * capr;   // this workgroup's part
    const bool overflowed = used > capr;   // else no sub-chunk of the part is flagged for it
    const unsigned long long nchunk = (cnt + 63) / 64;
    int n1 = 0;   // wave-uniform
    const uint64_t below = (1ull << lane) - 1;
    for (unsigned long long ch = (unsigned long long)(blockIdx.x / kQueueParts) * kDefWaves + wv;;
         ch += (unsigned long long)(gridDim.x / kQueueParts) * kDefWaves) {
        const bool tail = ch >= nchunk;
        while (n1 >= 64 || (tail && n1 > 0)) {   // resumed bins, 64 at a time
            wave_lds_sync();   // stack entries written by other lanes
            const int c = min(n1, 64);
            if (lane < c) {
                const uint32_t idx = S1[n1 - c + lane];
                const DeferredBin db = pq[idx];
                int next = 0;
                const float v = deferred_draw<MODE, kStageResume>(one, items, db, &next);
                if (v != v) defer_hard(pq, idx, next >= kNextFast ? next - kNextFast : next);
                else if (v != 0.f) deferred_add(one, items, db, v);
            }
            n1 -= c;
        }
        if (tail) break;
        const unsigned long long i = ch * 64 + lane;
        bool resume = false;
        if (i < cnt) {
            const DeferredBin db = pq[i];
            const RasterItem& I = items ? items[db.item & (kInvMark - 1u)] : one;
            if (db.depo != kInvalid && !(db.item & kHardMark) &&
                !(overflowed && (flags[I.sub_begin + db.depo / kSub] & kFlagOverflow))) {
                int next = 0;
                const float v = deferred_draw<MODE, kStageSecond>(one, items, db, &next);
                if (v != v) {
                    if (next >= kNextFast) resume = true;      // first try rejected
                    else defer_hard(pq, (uint32_t)i, next);  // log-scale test
                } else if (v != 0.f) {
                    deferred_add(one, items, db, v);
                }
            }
        }
        const uint64_t mm = __ballot(resume);
        if (resume) S1[n1 + __popcll(mm & below)] = (uint32_t)i;
        n1 += __popcll(mm);
    }
}

// The bins k_raster_deferred marked: the full rejection samplers, one try
// per pass, from the marked try.  Each wave scans 64 queue entries at a
// time and collects the marked ones in a wave-local stack; a batch of 64
// runs one full try of each (log-scale test included), and a bin whose try
// is rejected goes back on the stack with the next try.  The scan reads
// kScan chunks at a time so that their loads overlap.  (Running each bin
// to its end in one pass kept a wave busy for the longest lane's several
// tries.)  Inversion bins (queued by k_raster) take the full inversion;
// those of a sub-chunk whose later bins overflowed the queue are skipped, as
// k_raster_flagged redraws every deferred bin of such a sub-chunk.
template <int MODE>
__global__ __launch_bounds__(kDefWaves * 64) void k_raster_hard(RasterItem one,
                                                               const RasterItem* __restrict__ items,
                                                               const RasterWs* __restrict__ ws,
                                                               const uint8_t* __restrict__ flags,
                                                               const DeferredBin* __restrict__ queue,
                                                               unsigned long long cap) {
    constexpr int kScan = 4;                 // chunks of 64 entries scanned per step
    __shared__ uint32_t s_idx[kDefWaves][64 * (kScan + 2)];
    __shared__ uint16_t s_try[kDefWaves][64 * (kScan + 2)];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* SI = s_idx[wv];
    uint16_t* ST = s_try[wv];
    const unsigned part = blockIdx.x % kQueueParts;
    const unsigned long long capr = cap / kQueueParts, used = ws->count[part].v;
    const unsigned long long cnt = min(used, capr);
    const DeferredBin* const pq = queue + part * capr;   // this workgroup's part
    const bool overflowed = used > capr;   // else no sub-chunk of the part is flagged for it
    const unsigned long long nchunk = (cnt + 63) / 64;
    const uint64_t below = (1ull << lane) - 1;
    int n = 0;   // wave-uniform
    unsigned long long ch = (unsigned long long)(blockIdx.x / kQueueParts) * kDefWaves + wv;
    for (;;) {
        const bool tail = ch >= nchunk;
        if (n >= 64 || (tail && n > 0)) {
            wave_lds_sync();
            const int c = min(n, 64);
            bool again = false;
            uint32_t idx = 0;
            int t = 0;
            if (lane < c) {
                idx = SI[n - c + lane];
                t = ST[n - c + lane];
                DeferredBin db = pq[idx];
                const bool inv = (db.item & kInvMark) != 0u;
                db.item &= kInvMark - 1u;
                const RasterItem& I = items ? items[db.item] : one;
                const RasterArgs& A = I.A;
                if (!(overflowed && (flags[I.sub_begin + db.depo / kSub] & kFlagOverflow))) {
                    const float q = I.q[db.depo];
                    const float v = inv ? bin_count_in<false>(MODE, q, (double)db.p, A.seed, db.depo,
                                                              A.event, db.bin, A.plane)
                                        : bin_count_in<true>(MODE, q, (double)db.p, A.seed, db.depo,
                                                             A.event, db.bin, A.plane, t, t + 1);
                    if (v != v) again = true;
                    else if (v != 0.f) deferred_add(one, items, db, v);
                }
            }
            n -= c;
            const uint64_t mm = __ballot(again);
            if (again) {
                const int slot = n + __popcll(mm & below);
                SI[slot] = idx;
                ST[slot] = (uint16_t)(t + 1);
            }
            n += __popcll(mm);
            continue;
        }
        if (tail) break;
        // scan kScan chunks (their loads in flight together); n < 64 here,
        // so up to 64 * kScan more entries fit
        const unsigned long long G = (unsigned long long)(gridDim.x / kQueueParts) * kDefWaves;
        uint32_t item[kScan];
#pragma unroll
        for (int u = 0; u < kScan; ++u) {
            const unsigned long long i = (ch + u * G) * 64 + lane;
            item[u] = i < cnt ? pq[i].item : 0u;
        }
#pragma unroll
        for (int u = 0; u < kScan; ++u) {
            const unsigned long long i = (ch + u * G) * 64 + lane;
            const bool marked = (item[u] & kHardMark) != 0u;
            const uint64_t mm = __ballot(marked);
            if (marked) {
                const int slot = n + __popcll(mm & below);
                SI[slot] = (uint32_t)i;
                ST[slot] = (uint16_t)((item[u] >> kHardTryShift) & 7u);
            }
            n += __popcll(mm);
        }
        ch += kScan * G;
    }
}

// Flagged sub-chunks of a fluctuated raster.  A workgroup reads the flag
// bytes of 256 consecutive sub-chunks at once (one per thread) and takes the
// flagged ones in turn, one cell per thread:
//   kFlagWide      its depos wider than k_raster's weight slots: every bin,
//                  with weights per cell and the one-shot sampler;
//   kFlagOverflow  its regular depos' deferred bins (rejection-regime bins
//                  that the first try's immediate acceptance did not decide,
//                  inversion bins whose search ran off its end), recognised
//                  by redrawing the fast stage, then drawn with the full
//                  samplers; k_raster_deferred and k_raster_hard skip them.
template <int MODE>
__global__ __launch_bounds__(256) void k_raster_flagged(RasterItem one, const RasterItem* __restrict__ items,
                                                        int n_items, int64_t total_sub,
                                                        const uint8_t* __restrict__ flags) {
    __shared__ int s_list[256];
    __shared__ int s_n;
    for (int64_t g0 = (int64_t)blockIdx.x * 256; g0 < total_sub; g0 += (int64_t)gridDim.x * 256) {
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        const int64_t g = g0 + threadIdx.x;
        if (g < total_sub && flags[g]) s_list[atomicAdd(&s_n, 1)] = (int)threadIdx.x;
        __syncthreads();
        const int nf = s_n;
        for (int f = 0; f < nf; ++f) {
            const int64_t gsub = g0 + s_list[f];
            const int fl = flags[gsub];
            const RasterItem& I = items ? items[item_of(items, n_items, gsub)] : one;
            const RasterArgs& A = I.A;
            const int64_t sub = gsub - I.sub_begin;
            for (int dd = 0; dd < kSub; ++dd) {
                const int64_t gd = sub * kSub + dd;
                if (gd >= I.n) break;
                const float q = I.q[gd], t = I.t[gd], x = I.x[gd], st = I.st[gd], sx = I.sx[gd];
                if (!depo_finite(q, t, x, st, sx)) continue;
                const Window wt = axis_window(t, st, A.nsig, A.org_t, A.wd_t, A.n_ticks);
                if (!wt.n) continue;
                const Window wx = axis_window(x, sx, A.nsig, A.org_x, A.wd_x, A.n_rows);
                if (!wx.n) continue;
                const bool wide = wt.n > kMaxT || wx.n > kMaxX;
                if (!(fl & (wide ? kFlagWide : kFlagOverflow))) continue;
                const int64_t ncell = (int64_t)wt.n * wx.n;
                for (int64_t c = threadIdx.x; c < ncell; c += blockDim.x) {
                    const int a = (int)(c / wt.n), b = (int)(c - (int64_t)a * wt.n);
                    const float wtv = single_weight(t, st, A.org_t, A.wd_t, wt, b);
                    const float wxv = single_weight(x, sx, A.org_x, A.wd_x, wx, a);
                    const int j = wt.lo + b, m = wx.lo + a;
                    const double p = (double)(wtv * wxv);
                    const uint32_t bin = (uint32_t)((int64_t)m * A.n_ticks + j);
                    float v;
                    if (wide) {
                        v = bin_count(MODE, q, p, A.seed, (uint32_t)gd, A.event, bin, A.plane);
                    } else if constexpr (MODE == 3) {
                        continue;   // (mode 3 queues nothing: only wide depos are flagged)
                    } else {
                        // the bins k_raster queued: rejection bins the first stage
                        // left, inversion bins whose one-try search ran off its end
                        const bool rej = sampler_stack(MODE, q, p) == kStkF;
                        v = rej ? bin_count_fast<MODE, kStageFirst>(q, p, A.seed, (uint32_t)gd, A.event, bin,
                                                                    A.plane)
                                : bin_count_fast<MODE, kStageInv>(q, p, A.seed, (uint32_t)gd, A.event, bin,
                                                                  A.plane);
                        if (v == v) continue;   // drawn (and added) by k_raster
                        v = rej ? bin_count_in<true>(MODE, q, p, A.seed, (uint32_t)gd, A.event, bin, A.plane)
                                : bin_count_in<false>(MODE, q, p, A.seed, (uint32_t)gd, A.event, bin, A.plane);
                    }
                    if (v != 0.f) grid_add(&I.grid[(int64_t)m * A.ld + j], v);
                }
            }
        }
        __syncthreads();
    }
}

// Mean raster: depos whose window exceeds the weight slots of k_raster (kMaxT
// ticks or kMaxX impact rows): a workgroup scans kRasterThreads / kSub sub-chunks,
// one depo slot per thread, and processes the wide depos cooperatively, one
// cell per thread with weights per cell.  (Fluctuated rasters flag such
// sub-chunks in k_raster and take them in k_raster_flagged.)
__global__ __launch_bounds__(kRasterThreads) void k_raster_wide(RasterItem one,
                                                                const RasterItem* __restrict__ items,
                                                                int n_items, int64_t total_sub) {
    __shared__ int s_list[kRasterThreads];
    __shared__ int s_n;
    constexpr int SUBS = kRasterThreads / kSub;
    const int tid = threadIdx.x;
    for (int64_t g0 = (int64_t)blockIdx.x * SUBS; g0 < total_sub; g0 += (int64_t)gridDim.x * SUBS) {
        if (tid == 0) s_n = 0;
        __syncthreads();
        const int64_t gsub = g0 + tid / kSub;
        if (gsub < total_sub) {
            const RasterItem& I = items ? items[item_of(items, n_items, gsub)] : one;
            const RasterArgs& A = I.A;
            const int64_t d = (gsub - I.sub_begin) * kSub + tid % kSub;
            if (d < I.n) {
                const float q = I.q[d], t = I.t[d], x = I.x[d], st = I.st[d], sx = I.sx[d];
                if (depo_finite(q, t, x, st, sx)) {
                    const Window wt = axis_window(t, st, A.nsig, A.org_t, A.wd_t, A.n_ticks);
                    const Window wx = wt.n ? axis_window(x, sx, A.nsig, A.org_x, A.wd_x, A.n_rows)
                                           : Window{0, 0, false};
                    if (wt.n && wx.n && (wt.n > kMaxT || wx.n > kMaxX)) s_list[atomicAdd(&s_n, 1)] = tid;
                }
            }
        }
        __syncthreads();
        const int nw = s_n;
        for (int i = 0; i < nw; ++i) {
            const int slot = s_list[i];
            const int64_t gsub = g0 + slot / kSub;
            const RasterItem& I = items ? items[item_of(items, n_items, gsub)] : one;
            const RasterArgs& A = I.A;
            const int64_t gd = (gsub - I.sub_begin) * kSub + slot % kSub;
            const float q = I.q[gd], t = I.t[gd], x = I.x[gd], st = I.st[gd], sx = I.sx[gd];
            const Window wt = axis_window(t, st, A.nsig, A.org_t, A.wd_t, A.n_ticks);
            const Window wx = axis_window(x, sx, A.nsig, A.org_x, A.wd_x, A.n_rows);
            const int64_t ncell = (int64_t)wt.n * wx.n;
            for (int64_t c = tid; c < ncell; c += kRasterThreads) {
                const int a = (int)(c / wt.n), b = (int)(c - (int64_t)a * wt.n);
                const float wtv = single_weight(t, st, A.org_t, A.wd_t, wt, b);
                const float wxv = single_weight(x, sx, A.org_x, A.wd_x, wx, a);
                const int j = wt.lo + b, m = wx.lo + a;
                const float v = q * wtv * wxv;
                if (v != 0.f) grid_add(&I.grid[(int64_t)m * A.ld + j], v);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- skipped depos
//
// The depos every raster kernel skips (a non-finite field, depo_finite),
// counted into a device 64-bit counter: the counter is cleared by one
// thread of a one-block kernel, then each workgroup sums its wave counts in
// LDS and adds the total with one atomic (integer sums: the count does not
// depend on the order).
__global__ __launch_bounds__(64) void k_clear_count(unsigned long long* count) {
    if (threadIdx.x == 0) *count = 0ull;
}

__global__ __launch_bounds__(256) void k_count_nonfinite(const float* __restrict__ q, const float* __restrict__ t,
                                                         const float* __restrict__ x, const float* __restrict__ st,
                                                         const float* __restrict__ sx, int64_t n,
                                                         unsigned long long* __restrict__ count) {
    __shared__ unsigned s_part[4];
    unsigned c = 0;
    const int64_t step = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += step)
        c += depo_finite(q[i], t[i], x[i], st[i], sx[i]) ? 0u : 1u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned total = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        if (total) atomicAdd(count, (unsigned long long)total);
    }
}

hipError_t launch_count_nonfinite(const float* q, const float* t, const float* x, const float* st,
                                  const float* sx, int64_t n, int64_t* count, hipStream_t s) {
    unsigned long long* c = reinterpret_cast<unsigned long long*>(count);
    hipLaunchKernelGGL(k_clear_count, dim3(1), dim3(64), 0, s, c);
    if (n > 0) {
        const int64_t blocks = (n + 255) / 256, cap = 8 * (int64_t)device_cus();
        hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)(blocks < cap ? blocks : cap)), dim3(256), 0, s, q, t,
                           x, st, sx, n, c);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- adjoint raster
//
// Gradients of L = sum_{m,j} G[m][j] S[m][j] with respect to each depo's q,
// t, x, sigma_t, sigma_x for the mean patch, windows held fixed:
//   dw/dmu = -(phi(z_b) - phi(z_a))/sigma, dw/dsigma = -(z_b phi(z_b) - z_a phi(z_a))/sigma
// (phi the standard normal density).  One thread per depo recomputes its
// windows (same FP64 decisions as the forward raster) and weights, and
// gathers G over the patch row by row:
//   dq = sum_a wx_a r_a, dt = q sum_a wx_a s_a, dsigma_t = q sum_a wx_a u_a,
//   dx = q sum_a dwx_a r_a, dsigma_x = q sum_a dswx_a r_a
// with r_a, s_a, u_a the row's G sums weighted by wt, dwt/dmu, dwt/dsigma.

__device__ __forceinline__ float normal_pdf(float z) {
#pragma clang fp contract(off)
    return 0.39894228040143268f * expf(-0.5f * z * z);
}

// weight and its two derivatives for bin i of a window
__device__ __forceinline__ void weight_grads(double mu, double sg, double org, double wd,
                                             const Window& win, int i, float& w, float& dmu,
                                             float& dsg) {
    if (win.point) {
        w = 1.f; dmu = 0.f; dsg = 0.f;
        return;
    }
    const double inv = 1.0 / sg;
    const float za = edge_z(org, wd, win.lo + i, mu, inv);
    const float zb = edge_z(org, wd, win.lo + i + 1, mu, inv);
    w = bin_weight(za, zb, normal_tail(za), normal_tail(zb));
    const float pa = normal_pdf(za), pb = normal_pdf(zb);
    const float is = (float)inv;
    dmu = -(pb - pa) * is;
    dsg = -(zb * pb - za * pa) * is;
}

__global__ __launch_bounds__(256) void k_raster_bwd(RasterArgs A, const float* __restrict__ Q,
                                                    const float* __restrict__ Tm,
                                                    const float* __restrict__ X,
                                                    const float* __restrict__ ST,
                                                    const float* __restrict__ SX, int64_t n,
                                                    const float* __restrict__ G,
                                                    float* __restrict__ dq, float* __restrict__ dt,
                                                    float* __restrict__ dx, float* __restrict__ dst,
                                                    float* __restrict__ dsx) {
    constexpr int CH = 16;   // ticks per register chunk
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n;
         d += (int64_t)gridDim.x * blockDim.x) {
        float aq = 0.f, at = 0.f, ast = 0.f, ax = 0.f, asx = 0.f;
        const float q = Q[d], t = Tm[d], x = X[d], st = ST[d], sx = SX[d];
        if (depo_finite(q, t, x, st, sx)) {
            const Window wt = axis_window(t, st, A.nsig, A.org_t, A.wd_t, A.n_ticks);
            const Window wx = wt.n ? axis_window(x, sx, A.nsig, A.org_x, A.wd_x, A.n_rows)
                                   : Window{0, 0, false};
            for (int b0 = 0; b0 < wt.n && wx.n; b0 += CH) {
                float w[CH], wm[CH], ws[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    w[i] = wm[i] = ws[i] = 0.f;
                    if (b0 + i < wt.n) weight_grads(t, st, A.org_t, A.wd_t, wt, b0 + i, w[i], wm[i], ws[i]);
                }
                for (int a = 0; a < wx.n; ++a) {
                    float vx, vxm, vxs;
                    weight_grads(x, sx, A.org_x, A.wd_x, wx, a, vx, vxm, vxs);
                    const float* g = G + (int64_t)(wx.lo + a) * A.ld + wt.lo + b0;
                    float r = 0.f, sm = 0.f, ss = 0.f;
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        if (b0 + i < wt.n) {
                            const float gi = g[i];
                            r += gi * w[i];
                            sm += gi * wm[i];
                            ss += gi * ws[i];
                        }
                    }
                    aq += vx * r;
                    at += vx * sm;
                    ast += vx * ss;
                    ax += vxm * r;
                    asx += vxs * r;
                }
            }
        }
        dq[d] = aq;
        dt[d] = q * at;
        dst[d] = q * ast;
        dx[d] = q * ax;
        dsx[d] = q * asx;
    }
}

hipError_t launch_raster_bwd(const RasterArgs& a, const float* q, const float* t, const float* x,
                             const float* st, const float* sx, int64_t n, const float* grid_grad,
                             float* dq, float* dt, float* dx, float* dst, float* dsx, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256, cap = 16 * (int64_t)device_cus();
    hipLaunchKernelGGL(k_raster_bwd, dim3((unsigned)(blocks < cap ? blocks : cap)), dim3(256), 0, s, a,
                       q, t, x, st, sx, n, grid_grad, dq, dt, dx, dst, dsx);
    return hipGetLastError();
}

bool raster_tile_ok(int tile) { return tile == 384 || tile == 512 || tile == 640 || tile == 768; }

// X(T) with the compile-time tile T of a raster_tile_ok value
#define LAR_TILE_DISPATCH(tile, X)  \
    switch (tile) {                 \
        case 384: X(384) break;     \
        case 640: X(640) break;     \
        case 768: X(768) break;     \
        default: X(512) break;      \
    }

hipError_t launch_raster_items(int mode, const RasterItem& one, const RasterItem* items, int n_items,
                               int64_t total_sub, void* ws, size_t ws_bytes, hipStream_t s,
                               hipEvent_t main_done, int tile) {
    if (total_sub <= 0) return hipSuccess;
    if (!raster_tile_ok(tile)) return hipErrorInvalidValue;
    const int64_t cap_blocks = 8 * (int64_t)device_cus();
    const int64_t dgrid = kDeferredGroupsPerCU * (int64_t)device_cus();
    const int64_t nblk = (total_sub + kWaves - 1) / kWaves;
    const int64_t rcap = kRasterGroupsPerCU * (int64_t)device_cus();
    const dim3 grd((unsigned)(nblk < rcap ? nblk : rcap)), blk(kRasterThreads);
    const int64_t nwide = (total_sub + (kRasterThreads / kSub) - 1) / (kRasterThreads / kSub);
    dim3 gw((unsigned)(nwide < cap_blocks ? nwide : cap_blocks));
    if (mode == 0) {
#define LAR_MEAN(T)                                                                                     \
    hipLaunchKernelGGL((k_raster<0, T>), grd, blk, 0, s, one, items, n_items, total_sub, nullptr, nullptr, \
                       nullptr, 0ull);
        LAR_TILE_DISPATCH(tile, LAR_MEAN)
#undef LAR_MEAN
        if (main_done) (void)hipEventRecord(main_done, s);
        hipLaunchKernelGGL(k_raster_wide, gw, blk, 0, s, one, items, n_items, total_sub);
        return hipGetLastError();
    }
    const size_t fixed = raster_ws_fixed_subs(total_sub);
    RasterWs* hdr = reinterpret_cast<RasterWs*>(ws);
    uint8_t* flags = reinterpret_cast<uint8_t*>(ws) + 256;
    DeferredBin* queue = reinterpret_cast<DeferredBin*>(reinterpret_cast<char*>(ws) + fixed);
    // queue positions are 32-bit in k_raster_deferred's stacks
    const unsigned long long cap =
        std::min<unsigned long long>((ws_bytes - fixed) / sizeof(DeferredBin), 0xFFFFFFFFull);
    const int64_t rblk = (total_sub + 255) / 256;
    const dim3 g256((unsigned)(rblk < cap_blocks ? rblk : cap_blocks));   // 256 sub-chunks per block
    hipLaunchKernelGGL(k_raster_reset, g256, dim3(256), 0, s, hdr, flags, total_sub);
#define LAR_MAIN(T) \
    hipLaunchKernelGGL((k_raster<LAR_M, T>), grd, blk, 0, s, one, items, n_items, total_sub, hdr, flags, queue, cap);
#define LAR_FLUCT(M)                                                                                 \
    LAR_TILE_DISPATCH(tile, LAR_MAIN)                                                                \
    if (main_done) (void)hipEventRecord(main_done, s);                                               \
    hipLaunchKernelGGL(k_raster_deferred<M>, dim3((unsigned)dgrid), dim3(kDefWaves * 64), 0, s,       \
                       one, items, hdr, flags, queue, cap);                                          \
    hipLaunchKernelGGL(k_raster_hard<M>, dim3((unsigned)dgrid), dim3(kDefWaves * 64), 0, s, one,       \
                       items, hdr, flags, queue, cap);                                               \
    hipLaunchKernelGGL(k_raster_flagged<M>, g256, dim3(256), 0, s, one, items, n_items, total_sub, flags);
    if (mode == 1) {
#define LAR_M 1
        LAR_FLUCT(1)
#undef LAR_M
    } else if (mode == 2) {
#define LAR_M 2
        LAR_FLUCT(2)
#undef LAR_M
    } else {
        // normal approximation: no queued draws, only depos wider than the
        // weight slots are flagged
#define LAR_M 3
        LAR_TILE_DISPATCH(tile, LAR_MAIN)
#undef LAR_M
        if (main_done) (void)hipEventRecord(main_done, s);
        hipLaunchKernelGGL(k_raster_flagged<3>, g256, dim3(256), 0, s, one, items, n_items, total_sub, flags);
    }
#undef LAR_FLUCT
#undef LAR_MAIN
    return hipGetLastError();
}
#undef LAR_TILE_DISPATCH

hipError_t launch_raster(const RasterArgs& a, const float* q, const float* t, const float* x,
                         const float* st, const float* sx, int64_t n, float* grid, void* ws,
                         size_t ws_bytes, hipStream_t s, hipEvent_t main_done, int tile) {
    if (n <= 0) return hipSuccess;
    RasterItem one;
    one.A = a;
    one.q = q; one.t = t; one.x = x; one.st = st; one.sx = sx;
    one.grid = grid;
    one.n = n;
    one.sub_begin = 0;
    return launch_raster_items(a.mode, one, nullptr, 1, raster_subchunks(n), ws, ws_bytes, s, main_done, tile);
}

}  // namespace lar
