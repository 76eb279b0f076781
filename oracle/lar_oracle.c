/*
 * lar_oracle.c -- plain, slow, FP64 CPU oracle for the LArTPC signal
 * simulation hot path (Dong et al., "Evaluation of Portable Programming
 * Models to Accelerate LArTPC Detector Simulations", arXiv:2203.02479).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests and the benchmark's CPU-baseline
 * leg can check the GPU path against a direct transcription of the
 * definitions.  It shares no code, header, table or constant with the GPU
 * library.  Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared -lm.
 *
 * What it computes (paper Sec. 2.1 Eq. (1) first term; Sec. 2.2 "Raster",
 * "Scatter-add"; Sec. 3.1 binomial fluctuation of the reference code):
 *
 *  - Bins: tick j covers [t0 + j*tick, t0 + (j+1)*tick); impact row m covers
 *    [xl + m*d, xl + (m+1)*d) with xl = x0 - pitch/2 and d = pitch/n_imp.
 *  - Window: every bin that intersects [mu - ns*sigma, mu + ns*sigma], i.e.
 *    lo = floor((mu - ns*sigma - origin)/width), hi likewise with +, clipped
 *    to the grid.  sigma < 1e-6*width is a point charge in the bin holding mu.
 *  - Weights: w_j = Phi(z_{j+1}) - Phi(z_j), z = (edge - mu)/sigma, with the
 *    standard normal CDF Phi; no renormalisation over the window.
 *  - Mean grid: S[m][j] += q * wt[j] * wx[m].
 *  - Fluctuated grid: n ~ Binomial(rint|q|, wt*wx) (mode 1) or
 *    Poisson(|q|*wt*wx) (mode 2) drawn independently per bin, S += sign(q)*n.
 *    Uniforms come from Philox4x32-10 (Salmon et al., SC'11) with key
 *    (seed_lo, seed_hi) and counter (depo, event, m*n_ticks + j,
 *    plane*2^24 + draw), two 52-bit uniforms per block.  Binomial:
 *    inversion when n*min(p,1-p) < 10, else BTRD (Hormann 1993, "The
 *    generation of binomial random variates").
 *    Poisson: inversion when lambda < 10, else PTRS (Hormann 1993, "The
 *    transformed rejection method for generating Poisson random variables").
 *    Mode 3: the normal approximation of the binomial (Sec. 3.1), rounded
 *    to the nearest integer and clipped to [0, rint|q|].
 *  - Noise normals: Gaussian pairs per (wire, frequency) for the noise term
 *    N(t,x) of Eq. (1), from the same Philox stream layout in its own
 *    counter domain.
 *  - Adjoint raster: gradients of sum(G*S) with respect to q, t, x, sigma_t,
 *    sigma_x with the windows held fixed.
 *  - Brute-force convolution: M[w][t] = sum_k sum_dw sum_tau
 *    r[k][dw][tau] * S[((w-dw) mod Wf)*n_imp + k][(t - tau) mod Tf], with S
 *    zero on rows >= n_wires*n_imp and ticks >= n_ticks (circular in both
 *    axes over the FFT lengths, exactly what the FFT product computes).
 *
 * All floating point is FP64 with contraction off; inputs are the float32
 * arrays the GPU receives, widened exactly.  The loops over depositions run
 * on OpenMP threads (lo_set_threads; 1 by default): each thread takes whole
 * depositions and adds to the shared grid with atomic updates, so only the
 * order of the FP64 sums depends on the thread count (fluctuated counts are
 * integers and sum exactly).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LO_SQRT1_2 0.70710678118654752440
#define LO_INV_SQRT2PI 0.39894228040143267794

/* ------------------------------------------------------------ Gaussian bins */

/* Standard normal density. */
static double lo_pdf(double z) { return LO_INV_SQRT2PI * exp(-0.5 * z * z); }

/* Phi(zb) - Phi(za) for za <= zb, each term written with the erfc of the side
 * away from the mean so that tails keep their relative precision. */
double lo_phi_diff(double za, double zb)
{
    if (za >= 0.0)
        return 0.5 * (erfc(za * LO_SQRT1_2) - erfc(zb * LO_SQRT1_2));
    if (zb <= 0.0)
        return 0.5 * (erfc(-zb * LO_SQRT1_2) - erfc(-za * LO_SQRT1_2));
    return 1.0 - 0.5 * erfc(zb * LO_SQRT1_2) - 0.5 * erfc(-za * LO_SQRT1_2);
}

/* One axis of a deposition: window [lo, lo+n) over nbins bins of `width`
 * starting at `origin`, weights w[] and (optionally) their derivatives with
 * respect to the centre mu and the width sigma.  Returns n (0 = no overlap). */
int lo_axis(double mu, double sigma, double nsig, double origin, double width,
            int nbins, int *lo_out, double *w, double *dmu, double *dsig)
{
    if (sigma < 1e-6 * width) {           /* point charge */
        double f = floor((mu - origin) / width);
        if (!(f >= 0.0) || f >= (double)nbins) return 0;
        *lo_out = (int)f;
        w[0] = 1.0;
        if (dmu) dmu[0] = 0.0;
        if (dsig) dsig[0] = 0.0;
        return 1;
    }
    double flo = floor((mu - nsig * sigma - origin) / width);
    double fhi = floor((mu + nsig * sigma - origin) / width);
    if (flo < 0.0) flo = 0.0;
    if (fhi > (double)(nbins - 1)) fhi = (double)(nbins - 1);
    if (!(flo <= fhi)) return 0;
    int lo = (int)flo, hi = (int)fhi;
    for (int j = lo; j <= hi; ++j) {
        double ea = origin + (double)j * width;
        double eb = origin + (double)(j + 1) * width;
        double za = (ea - mu) / sigma;
        double zb = (eb - mu) / sigma;
        w[j - lo] = lo_phi_diff(za, zb);
        if (dmu) dmu[j - lo] = -(lo_pdf(zb) - lo_pdf(za)) / sigma;
        if (dsig) dsig[j - lo] = -(zb * lo_pdf(zb) - za * lo_pdf(za)) / sigma;
    }
    *lo_out = lo;
    return hi - lo + 1;
}

static int lo_finite5(float a, float b, float c, float d, float e)
{
    return isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d) && isfinite(e);
}

typedef struct {
    int nt, nx, jlo, mlo;
    double *wt, *wx, *dwt_dmu, *dwt_ds, *dwx_dmu, *dwx_ds;
} lo_patch;

/* Windows and weights of depo i on a plane (both axes). */
static int lo_make_patch(int n_rows, int n_ticks, double pitch, double x0, int n_imp,
                         double tick, double t0, double nsig, double t, double x,
                         double st, double sx, lo_patch *P, int want_deriv)
{
    double xl = x0 - pitch / 2.0;
    double d = pitch / (double)n_imp;
    P->nt = lo_axis(t, st, nsig, t0, tick, n_ticks, &P->jlo, P->wt,
                    want_deriv ? P->dwt_dmu : NULL, want_deriv ? P->dwt_ds : NULL);
    if (P->nt == 0) return 0;
    P->nx = lo_axis(x, sx, nsig, xl, d, n_rows, &P->mlo, P->wx,
                    want_deriv ? P->dwx_dmu : NULL, want_deriv ? P->dwx_ds : NULL);
    return P->nx;
}

static int lo_alloc_patch(lo_patch *P, int n_ticks, int n_rows)
{
    P->wt = malloc(sizeof(double) * (size_t)n_ticks * 3);
    P->wx = malloc(sizeof(double) * (size_t)n_rows * 3);
    if (!P->wt || !P->wx) { free(P->wt); free(P->wx); return -1; }
    P->dwt_dmu = P->wt + n_ticks; P->dwt_ds = P->wt + 2 * (size_t)n_ticks;
    P->dwx_dmu = P->wx + n_rows; P->dwx_ds = P->wx + 2 * (size_t)n_rows;
    return 0;
}

static void lo_free_patch(lo_patch *P) { free(P->wt); free(P->wx); }

/* Mean grid S[m][j] += q*wt[j]*wx[m] over all depos (grid accumulates). */
int lo_raster_mean(int n_wires, int n_imp, int n_ticks, double pitch, double x0,
                   double tick, double t0, double nsig, int64_t n,
                   const float *q, const float *t, const float *x,
                   const float *st, const float *sx, double *grid)
{
    int n_rows = n_wires * n_imp;
    int failed = 0;
#pragma omp parallel reduction(| : failed)
    {
        lo_patch P;
        if (lo_alloc_patch(&P, n_ticks, n_rows)) {
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < n; ++i) {
                if (!lo_finite5(q[i], t[i], x[i], st[i], sx[i])) continue;
                if (!lo_make_patch(n_rows, n_ticks, pitch, x0, n_imp, tick, t0, nsig,
                                   t[i], x[i], st[i], sx[i], &P, 0)) continue;
                double qi = q[i];
                for (int a = 0; a < P.nx; ++a) {
                    double *row = grid + (size_t)(P.mlo + a) * n_ticks + P.jlo;
                    for (int b = 0; b < P.nt; ++b) {
                        double v = qi * P.wt[b] * P.wx[a];
#pragma omp atomic
                        row[b] += v;
                    }
                }
            }
            lo_free_patch(&P);
        }
    }
    return failed ? -1 : 0;
}

/* Threads of the depo loops (omp_set_num_threads); returns the count set. */
int lo_set_threads(int n)
{
    if (n < 1) n = 1;
    omp_set_num_threads(n);
    return n;
}

/* ------------------------------------------------------------ Philox4x32-10 */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): each round multiplies words 0 and 2
 * by the two round multipliers, swaps halves and mixes in the key, and the
 * key is bumped by the Weyl constants between rounds. */
void lo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream of uniforms for one bin: two 53-bit uniforms per Philox block, the
 * last counter word = plane*2^24 + draw, draw incremented per block. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int left;                   /* uniforms left in buf: 2, 1 or 0 */
} lo_stream;

static void lo_stream_init(lo_stream *s, uint64_t seed, uint32_t depo, uint32_t event,
                           uint32_t bin, uint32_t plane)
{
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    s->ctr[0] = depo; s->ctr[1] = event; s->ctr[2] = bin;
    s->ctr[3] = plane << 24;
    s->left = 0;
}

/* u = ((a >> 6) * 2^26 + (b >> 6) + 1/2) * 2^-52: a 52-bit integer plus one
 * half, scaled exactly, so u lies in [2^-53, 1 - 2^-53], strictly inside (0, 1). */
double lo_u53(uint32_t a, uint32_t b)
{
    double hi = (double)(a >> 6);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 4503599627370496.0);
}

static double lo_uniform(lo_stream *s)
{
    if (s->left == 0) {
        lo_philox4x32_10(s->ctr, s->key, s->buf);
        s->ctr[3] += 1u;
        s->left = 2;
        return lo_u53(s->buf[0], s->buf[1]);
    }
    s->left = 0;
    return lo_u53(s->buf[2], s->buf[3]);
}

/* ------------------------------------------------------------ samplers */

#define LO_MAX_TRIES 1000

/* log(k!) - [(k + 1/2) log(k+1) - (k+1) + log(2 pi)/2]: exact via lgamma for
 * small k, Stirling series (three terms) above. */
double lo_fc(double k)
{
    if (k < 10.0)
        return lgamma(k + 1.0) - (k + 0.5) * log(k + 1.0) + (k + 1.0)
               - 0.91893853320467274178;
    double r = 1.0 / (k + 1.0);
    double r2 = r * r;
    return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * r2) * r2) * r;
}

/* x^n for a non-negative integer n (held in a double) by binary powering:
 * square-and-multiply over the bits of n from the least significant. */
static double lo_ipow(double x, double n)
{
    uint64_t e = (uint64_t)n;
    double r = 1.0, b = x;
    while (e) {
        if (e & 1u) r = r * b;
        e >>= 1;
        if (e) b = b * b;
    }
    return r;
}

/* Binomial(n, p) by sequential inversion from k = 0 (p <= 1/2, n*p < 10):
 * f(0) = (1-p)^n, f(k) = f(k-1) * (g * (1/k) - r) with r = p/(1-p),
 * g = (n+1) r and 1/k the correctly rounded reciprocal. */
static double lo_binom_inv(double n, double p, lo_stream *s)
{
    double q = 1.0 - p;
    double ratio = p / q;
    double g = ratio * (n + 1.0);
    double f0 = lo_ipow(q, n);
    for (int tries = 0; tries < LO_MAX_TRIES; ++tries) {
        double u = lo_uniform(s);
        double f = f0;
        double k = 0.0;
        for (;;) {
            if (u < f) return k;
            if (k >= n || k > 110.0) break;       /* numerical tail: redraw */
            u = u - f;
            k = k + 1.0;
            f = f * (g * (1.0 / k) - ratio);
        }
    }
    return floor(n * p);
}

/* BTRD's test for a try far from the mode (|k - m| > 15): accept when
 * log v <= log f(k) - log f(m), first through the squeeze bounds t -+ rho of
 * that log ratio, then through its Stirling form with the corrections fc. */
static int lo_btrd_log_test(double v, double k, double n, double m, double r, double npq)
{
    double km = fabs(k - m);
    v = log(v);                               /* squeeze on log scale */
    double rho = (km / npq) * (((km / 3.0 + 0.625) * km + 1.0 / 6.0) / npq + 0.5);
    double t = -km * km / (2.0 * npq);
    if (v < t - rho) return 1;
    if (v > t + rho) return 0;
    double nm = n - m + 1.0;
    double h = (m + 0.5) * log((m + 1.0) / (r * nm)) + lo_fc(m) + lo_fc(n - m);
    double nk = n - k + 1.0;
    return v <= h + (n + 1.0) * log(nm / nk) + (k + 0.5) * log(nk * r / (k + 1.0))
                - lo_fc(k) - lo_fc(n - k);
}

/* Binomial(n, p) by BTRD (p <= 1/2, n*p >= 10). */
static double lo_binom_btrd(double n, double p, lo_stream *s)
{
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
    for (int tries = 0; tries < LO_MAX_TRIES; ++tries) {
        double v = lo_uniform(s);
        double u;
        if (v <= urvr) {                          /* fast acceptance region */
            u = v / vr - 0.43;
            return floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
        }
        if (v >= vr) {
            u = lo_uniform(s) - 0.5;
        } else {
            u = v / vr - 0.93;
            u = copysign(0.5, u) - u;
            v = lo_uniform(s) * vr;
        }
        double us = 0.5 - fabs(u);
        double k = floor((2.0 * a / us + b) * u + c);
        if (k < 0.0 || k > n) continue;
        v = v * alpha / (a / (us * us) + b);
        double km = fabs(k - m);
        if (km <= 15.0) {
            /* explicit pmf ratio f(k)/f(m) = prod (nr/i - r), as the product
             * of the numerators (nr - r i) over the product of the i's */
            double num = 1.0, den = 1.0;
            if (m < k) {
                for (double i = m + 1.0; i <= k; i = i + 1.0) { num = num * (nr - r * i); den = den * i; }
                if (v * den <= num) return k;
            } else if (m > k) {
                for (double i = k + 1.0; i <= m; i = i + 1.0) { num = num * (nr - r * i); den = den * i; }
                if (v * num <= den) return k;
            } else if (v <= 1.0) {
                return k;
            }
            continue;
        }
        if (lo_btrd_log_test(v, k, n, m, r, npq)) return k;
    }
    return m;
}

/* BTRD's acceptance decision for a try with |k - m| > 15 (v: the try's
 * rescaled uniform), without the standalone setup of lo_binom_btrd; exported
 * so that tests can compare it with the exact pmf ratio. */
int lo_btrd_log_accept(double n, double p, double k, double v)
{
    double m = floor((n + 1.0) * p);
    double r = p / (1.0 - p);
    double npq = n * p * (1.0 - p);
    return lo_btrd_log_test(v, k, n, m, r, npq);
}

/* Binomial(n, p) for any p in [0, 1]. */
double lo_binomial(double n, double p, lo_stream *s)
{
    if (!(n > 0.0) || !(p > 0.0)) return 0.0;
    if (p >= 1.0) return n;
    int flip = p > 0.5;
    double pp = flip ? 1.0 - p : p;
    double k = (n * pp < 10.0) ? lo_binom_inv(n, pp, s) : lo_binom_btrd(n, pp, s);
    return flip ? n - k : k;
}

/* PTRS's final test: accept k when v, rescaled by the hat function at u
 * (alpha / (a/us^2 + b)), lies below the Poisson pmf at k, on a log scale. */
static int lo_ptrs_log_test(double lam, double loglam, double a, double b, double invalpha,
                            double us, double v, double k)
{
    return log(v) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0);
}

/* Poisson(lambda): inversion below 10, PTRS above. */
double lo_poisson(double lam, lo_stream *s)
{
    if (!(lam > 0.0)) return 0.0;
    if (lam < 10.0) {
        double p0 = exp(-lam);
        for (int tries = 0; tries < LO_MAX_TRIES; ++tries) {
            double u = lo_uniform(s);
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
    for (int tries = 0; tries < LO_MAX_TRIES; ++tries) {
        double u = lo_uniform(s) - 0.5;
        double v = lo_uniform(s);
        double us = 0.5 - fabs(u);
        double k = floor((2.0 * a / us + b) * u + lam + 0.43);
        if (us >= 0.07 && v <= vr) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        if (lo_ptrs_log_test(lam, loglam, a, b, invalpha, us, v, k)) return k;
    }
    return floor(lam);
}

/* PTRS's final acceptance decision for candidate k from (u, v), lam >= 10,
 * with PTRS's setup constants; exported so that tests can compare it with
 * the exact Poisson pmf. */
int lo_ptrs_log_accept(double lam, double us, double v, double k)
{
    double b = 0.931 + 2.53 * sqrt(lam);
    double a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    return lo_ptrs_log_test(lam, log(lam), a, b, invalpha, us, v, k);
}

/* Standard normal deviates from two uniforms (Box and Muller 1958): the
 * cosine branch sqrt(-2 log u1) cos(2 pi u2) and the sine branch. */
void lo_box_muller(double u1, double u2, double *z_cos, double *z_sin)
{
    double r = sqrt(-2.0 * log(u1));
    double a = 6.283185307179586 * u2;
    *z_cos = r * cos(a);
    if (z_sin) *z_sin = r * sin(a);
}

/* Normal approximation of Binomial(n, p) (the GPU port's choice, Sec. 3.1):
 * mu = n p, sd = sqrt(mu (1 - p)), count = mu + sd z rounded to the nearest
 * integer (ties to even) and clipped to [0, n], with z the cosine branch of
 * Box-Muller on the bin's first two uniforms. */
double lo_binomial_normal(double n, double p, lo_stream *s)
{
    if (!(n > 0.0) || !(p > 0.0)) return 0.0;
    if (p >= 1.0) return n;
    double u1 = lo_uniform(s);
    double u2 = lo_uniform(s);
    double z;
    lo_box_muller(u1, u2, &z, NULL);
    double mu = n * p;
    double sd = sqrt(mu * (1.0 - p));
    double k = rint(mu + sd * z);
    if (k < 0.0) k = 0.0;
    if (k > n) k = n;
    return k;
}

/* Signed fluctuated count for one bin: sign(q) * n with n drawn for
 * mode 1 = Binomial(rint|q|, p), mode 2 = Poisson(|q| p), mode 3 = the
 * normal approximation of Binomial(rint|q|, p). */
double lo_bin_count(int mode, float q, double p, uint64_t seed, uint32_t depo,
                    uint32_t event, uint32_t bin, uint32_t plane)
{
    lo_stream s;
    lo_stream_init(&s, seed, depo, event, bin, plane);
    double aq = fabs((double)q);
    double n;
    if (mode == 1) n = lo_binomial(rint(aq), p, &s);
    else if (mode == 2) n = lo_poisson(aq * p, &s);
    else n = lo_binomial_normal(rint(aq), p, &s);
    return q < 0.0f ? -n : n;
}

/* Batch entry for tests: out[i] = lo_bin_count(mode, q[i], p[i], ctr[i]). */
void lo_sample_counts(int mode, int64_t n, const float *q, const double *p,
                      const uint32_t *ctr3, uint32_t plane, uint64_t seed, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = lo_bin_count(mode, q[i], p[i], seed, ctr3[3 * i], ctr3[3 * i + 1],
                              ctr3[3 * i + 2], plane);
}

/* Gaussian pairs of the noise term (Eq. (1) second term): for wire w and
 * frequency bin f, one Philox block with counter (w, event, f, plane*2^24 +
 * 2^23) -- bit 23 of the last word marks the noise domain, which the raster's
 * draw index never reaches -- gives two uniforms and Box-Muller's cosine and
 * sine branches, written to re[w*nf + f] and im[w*nf + f]. */
void lo_noise_normals(uint64_t seed, uint32_t event, uint32_t plane, int n_wires, int nf,
                      double *re, double *im)
{
    for (int w = 0; w < n_wires; ++w)
        for (int f = 0; f < nf; ++f) {
            lo_stream s;
            lo_stream_init(&s, seed, (uint32_t)w, event, (uint32_t)f, plane);
            s.ctr[3] += 0x00800000u;
            double u1 = lo_uniform(&s);
            double u2 = lo_uniform(&s);
            lo_box_muller(u1, u2, &re[(size_t)w * nf + f], &im[(size_t)w * nf + f]);
        }
}

/* Raw uniforms of one stream, for tests of the stream layout. */
void lo_stream_uniforms(uint64_t seed, uint32_t depo, uint32_t event, uint32_t bin,
                        uint32_t plane, int count, double *out)
{
    lo_stream s;
    lo_stream_init(&s, seed, depo, event, bin, plane);
    for (int i = 0; i < count; ++i) out[i] = lo_uniform(&s);
}

/* Fluctuated grid (accumulates): S[m][j] += sign(q) * n_{depo,m,j}. */
int lo_raster_fluct(int n_wires, int n_imp, int n_ticks, double pitch, double x0,
                    double tick, double t0, double nsig, int64_t n,
                    const float *q, const float *t, const float *x,
                    const float *st, const float *sx, int mode, uint64_t seed,
                    uint32_t event, uint32_t plane, double *grid)
{
    int n_rows = n_wires * n_imp;
    int failed = 0;
#pragma omp parallel reduction(| : failed)
    {
        lo_patch P;
        if (lo_alloc_patch(&P, n_ticks, n_rows)) {
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < n; ++i) {
                if (!lo_finite5(q[i], t[i], x[i], st[i], sx[i])) continue;
                if (!lo_make_patch(n_rows, n_ticks, pitch, x0, n_imp, tick, t0, nsig,
                                   t[i], x[i], st[i], sx[i], &P, 0)) continue;
                for (int a = 0; a < P.nx; ++a) {
                    int m = P.mlo + a;
                    for (int b = 0; b < P.nt; ++b) {
                        int j = P.jlo + b;
                        double p = P.wt[b] * P.wx[a];
                        uint32_t bin = (uint32_t)((int64_t)m * n_ticks + j);
                        double c = lo_bin_count(mode, q[i], p, seed, (uint32_t)i, event, bin, plane);
#pragma omp atomic
                        grid[(size_t)m * n_ticks + j] += c;
                    }
                }
            }
            lo_free_patch(&P);
        }
    }
    return failed ? -1 : 0;
}

/* ------------------------------------------------------------ adjoint raster */

/* Gradients of L = sum_{m,j} G[m][j] * S[m][j] (mean grid) with respect to the
 * depo parameters, windows held fixed. */
int lo_raster_adjoint(int n_wires, int n_imp, int n_ticks, double pitch, double x0,
                      double tick, double t0, double nsig, int64_t n,
                      const float *q, const float *t, const float *x,
                      const float *st, const float *sx, const double *G,
                      double *dq, double *dt, double *dx, double *dst, double *dsx)
{
    int n_rows = n_wires * n_imp;
    int failed = 0;
#pragma omp parallel reduction(| : failed)
    {
        lo_patch P;
        if (lo_alloc_patch(&P, n_ticks, n_rows)) {
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < n; ++i) {
                dq[i] = dt[i] = dx[i] = dst[i] = dsx[i] = 0.0;
                if (!lo_finite5(q[i], t[i], x[i], st[i], sx[i])) continue;
                if (!lo_make_patch(n_rows, n_ticks, pitch, x0, n_imp, tick, t0, nsig,
                                   t[i], x[i], st[i], sx[i], &P, 1)) continue;
                double s_q = 0, s_t = 0, s_st = 0, s_x = 0, s_sx = 0;
                for (int a = 0; a < P.nx; ++a) {
                    const double *row = G + (size_t)(P.mlo + a) * n_ticks + P.jlo;
                    for (int b = 0; b < P.nt; ++b) {
                        double g = row[b];
                        s_q += g * P.wt[b] * P.wx[a];
                        s_t += g * P.dwt_dmu[b] * P.wx[a];
                        s_st += g * P.dwt_ds[b] * P.wx[a];
                        s_x += g * P.wt[b] * P.dwx_dmu[a];
                        s_sx += g * P.wt[b] * P.dwx_ds[a];
                    }
                }
                double qi = q[i];
                dq[i] = s_q;
                dt[i] = qi * s_t;
                dst[i] = qi * s_st;
                dx[i] = qi * s_x;
                dsx[i] = qi * s_sx;
            }
            lo_free_patch(&P);
        }
    }
    return failed ? -1 : 0;
}

/* ------------------------------------------------------------ direct convolution */

/* Brute-force Eq. (1) first term on the discrete grid, circular over (Wf, Tf):
 * M[w][t] = sum_k sum_dw sum_tau r[k][dw+H][tau] * S[row(w-dw, k)][(t-tau) mod Tf].
 * r is [n_imp][2H+1][L]; S is [n_wires*n_imp][n_ticks]; M is [n_wires][n_ticks]. */
void lo_conv_direct(int n_wires, int n_imp, int n_ticks, int nw_fft, int nt_fft,
                    int half_w, int n_rt, const double *r, const double *S, double *M)
{
    for (int w = 0; w < n_wires; ++w)
        for (int tt = 0; tt < n_ticks; ++tt) {
            double acc = 0.0;
            for (int k = 0; k < n_imp; ++k)
                for (int dw = -half_w; dw <= half_w; ++dw) {
                    int ws = ((w - dw) % nw_fft + nw_fft) % nw_fft;
                    if (ws >= n_wires) continue;
                    const double *rk = r + ((size_t)k * (2 * half_w + 1) + (dw + half_w)) * n_rt;
                    const double *srow = S + (size_t)(ws * n_imp + k) * n_ticks;
                    for (int tau = 0; tau < n_rt; ++tau) {
                        int ts = ((tt - tau) % nt_fft + nt_fft) % nt_fft;
                        if (ts >= n_ticks) continue;
                        acc += rk[tau] * srow[ts];
                    }
                }
            M[(size_t)w * n_ticks + tt] = acc;
        }
}
