"""Pins of the oracle's normal-approximation sampler, drift stage, noise term
and digitiser against closed forms, exact distributions, Monte Carlo of the
physical process and finite differences.  CPU only."""
from fractions import Fraction
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import stages
from paper_2203_02479_amd import inputs


# ------------------------------------------------------------------ normal approximation (mode 3)

def _draw(mode, q, p, n, seed=91):
    ctr = np.zeros((n, 3), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 2
    ctr[:, 2] = 4321
    return oracle.sample_counts(mode, np.full(n, q, np.float32), np.full(n, p), ctr, 1, seed)


def _rounded_normal_pmf(N, p, ks):
    """Exact pmf of clip(rint(N p + sqrt(N p (1-p)) Z), 0, N), Z standard
    normal: the mass of each integer's rounding interval, with the tails
    lumped at 0 and N (ties have probability zero)."""
    mu, sd = N * p, math.sqrt(N * p * (1 - p))
    hi = stats.norm.cdf((ks + 0.5 - mu) / sd)
    lo = stats.norm.cdf((ks - 0.5 - mu) / sd)
    pmf = hi - lo
    pmf = np.where(ks == 0, hi, pmf)
    pmf = np.where(ks == N, 1.0 - lo, pmf)
    return np.where((ks < 0) | (ks > N), 0.0, pmf)


def _chi2_pvalue(samples, pmf, kmax):
    ks = np.arange(kmax + 1)
    expect = pmf(ks) * len(samples)
    obs = np.bincount(samples.astype(np.int64), minlength=kmax + 1)[:kmax + 1].astype(float)
    e_b, o_b, ce, co = [], [], 0.0, 0.0
    for e, o in zip(expect, obs):
        ce += e
        co += o
        if ce >= 5:
            e_b.append(ce)
            o_b.append(co)
            ce = co = 0.0
    if e_b:
        e_b[-1] += ce
        o_b[-1] += co
    e_b, o_b = np.array(e_b), np.array(o_b)
    e_b *= o_b.sum() / e_b.sum()
    chi2 = ((o_b - e_b) ** 2 / e_b).sum()
    return stats.chi2.sf(chi2, max(len(e_b) - 1, 1))


@pytest.mark.parametrize("N,p", [(1000, 0.3), (20, 0.05), (50, 0.97), (100000, 0.001), (5, 0.5),
                                 (2500, 0.7), (3, 0.2), (40, 0.5)])
def test_normal_approx_matches_exact_rounded_normal_pmf(N, p):
    s = _draw(3, float(N), p, 20000)
    assert s.min() >= 0 and s.max() <= N and np.all(s == np.round(s))
    kmax = N if N < 5000 else int(N * p + 12 * math.sqrt(N * p) + 12)
    pv = _chi2_pvalue(s, lambda k: _rounded_normal_pmf(N, p, k), kmax)
    assert pv > 1e-4, (N, p, pv)


def test_normal_approx_close_to_binomial_at_large_mean():
    """With no skew (p = 1/2) and a large mean, the approximation is
    indistinguishable from the binomial at this sample size; its variance is
    N p (1 - p) plus the rounding's 1/12."""
    N, p = 4000, 0.5
    s = _draw(3, float(N), p, 20000)
    pv = _chi2_pvalue(s, lambda k: stats.binom.pmf(k, N, p), N)
    assert pv > 1e-4
    assert abs(s.mean() - N * p) < 5 * math.sqrt(N * p * (1 - p) / len(s))
    assert s.var() == pytest.approx(N * p * (1 - p) + 1 / 12, rel=0.05)


def test_normal_approx_edges_and_sign():
    ctr = np.array([[i, 0, 0] for i in range(5)], np.uint32)
    out = oracle.sample_counts(3, np.array([-40.0, 40.0, 0.0, 7.0, -9.0], np.float32),
                               np.array([1.0, 0.0, 0.5, 1.0, 0.5]), ctr, 0, 3)
    assert list(out[:4]) == [-40.0, 0.0, 0.0, 7.0]
    assert out[4] <= 0 and out[4] >= -9


def test_normal_approx_uses_the_bins_first_block():
    """count = rint(mu + sd z) with z the cosine branch of Box-Muller on the
    stream's first two uniforms (one Philox block)."""
    seed, depo, ev, b, pl = 12345, 7, 1, 99, 3
    u = oracle.stream_uniforms(seed, depo, ev, b, pl, 2)
    z, _ = oracle.box_muller(u[0], u[1])
    N, p = 900.0, 0.21
    got = oracle.sample_counts(3, np.array([N], np.float32), np.array([p]),
                               np.array([[depo, ev, b]], np.uint32), pl, seed)[0]
    assert got == np.clip(np.rint(N * p + math.sqrt(N * p * (1 - p)) * z), 0, N)


def test_box_muller_closed_form_points():
    """u2 = 0 gives the cosine branch sqrt(-2 log u1); u2 = 1/4 moves it to
    the sine branch; u1 = exp(-1/2) gives radius 1."""
    c, s = oracle.box_muller(math.exp(-0.5), 0.0)
    assert c == pytest.approx(1.0, abs=1e-15) and s == 0.0
    c, s = oracle.box_muller(math.exp(-2.0), 0.25)
    assert s == pytest.approx(2.0, abs=1e-15) and abs(c) < 1e-15
    c, s = oracle.box_muller(0.5, 0.5)
    assert c == pytest.approx(-math.sqrt(2 * math.log(2)), rel=1e-15)


def test_fluctuated_grid_mode3_mean_and_variance():
    P = inputs.Plane(n_wires=6, n_ticks=40, n_imp=3, nt_fft=48, nw_fft=12, half_w=2)
    f = np.float32
    dep = inputs.Depos(*(np.array([v], f) for v in (4000.0, 9.3, 3.1, 0.6, 0.7)))
    mean = oracle.raster_mean(P, dep)
    reps = np.stack([oracle.raster_fluct(P, dep, mode=3, seed=s) for s in range(400)])
    big = mean > 30
    var_ref = mean * (1 - mean / 4000.0) + 1 / 12
    z = (reps.mean(0) - mean)[big] / np.sqrt(var_ref[big] / 400)
    assert np.abs(z).max() < 5.0
    np.testing.assert_allclose(reps.var(0)[big], var_ref[big], rtol=0.4)


# ------------------------------------------------------------------ drift

PARAMS = (inputs.V_DRIFT, inputs.D_L, inputs.D_T, 3000.0)
PROJ = np.array([[inputs.COS60, inputs.SIN60, 0.0], [inputs.COS60, -inputs.SIN60, 3000.0 * inputs.SIN60],
                 [1.0, 0.0, 0.0]])


def _groups(n, seed=3):
    rng = np.random.default_rng(seed)
    f = np.float32
    return (rng.uniform(100, 6000, n).astype(f), rng.uniform(0, 50, n).astype(f),
            rng.uniform(-20, 3600, n).astype(f), rng.uniform(0, 3000, n).astype(f),
            rng.uniform(0, 2400, n).astype(f))


def test_drift_zero_drift_is_identity():
    q0, t0, _, y, z = _groups(50)
    xd = np.concatenate([np.zeros(25), -np.abs(np.linspace(1, 9, 25))]).astype(np.float32)
    q, t, st, sx, x = oracle.drift(PARAMS, q0, t0, xd, y, z, PROJ)
    np.testing.assert_array_equal(q, q0.astype(np.float64))
    np.testing.assert_array_equal(t, t0.astype(np.float64))
    assert not st.any() and not sx.any()


def test_drift_brownian_motion_monte_carlo():
    """Diffusion as Brownian motion dX = sqrt(2 D) dW over the drift time: the
    spread of simulated electrons matches sigma_T (space) and sigma_L * v
    (time units) within their sampling error; the surviving fraction of
    electrons with exponential lifetimes matches the attenuation."""
    rng = np.random.default_rng(11)
    xd = 2400.0
    td = xd / np.float32(inputs.V_DRIFT)
    n_e, n_steps = 20000, 200
    dt = td / n_steps
    for D in (inputs.D_T, inputs.D_L):
        X = np.zeros(n_e)
        for _ in range(n_steps):
            X += math.sqrt(2.0 * float(np.float32(D)) * dt) * rng.standard_normal(n_e)
        q, t, st, sx, _ = oracle.drift(PARAMS, [1.0], [0.0], [xd], [0.0], [0.0], PROJ)
        want = sx[0] if D == inputs.D_T else st[0] * float(np.float32(inputs.V_DRIFT))
        assert X.std() == pytest.approx(want, rel=4 / math.sqrt(2 * n_e))
    life = rng.exponential(float(np.float32(PARAMS[3])), 200000)
    q, *_ = oracle.drift(PARAMS, [1.0], [0.0], [xd], [0.0], [0.0], PROJ)
    frac = np.mean(life > td)
    assert frac == pytest.approx(q[0], abs=4 * math.sqrt(q[0] * (1 - q[0]) / len(life)))


def test_drift_semigroup_and_linear_time():
    """Drifting d1 then d2 equals drifting d1 + d2: widths add in quadrature,
    attenuations multiply, arrival times add."""
    p64 = np.array(PARAMS, np.float64)
    one = lambda d: stages.drift_f64(p64, np.ones(1), np.zeros(1), np.array([d]), np.zeros(1), np.zeros(1), PROJ)
    a, b, ab = one(700.0), one(1300.0), one(2000.0)
    assert ab[3][0] ** 2 == pytest.approx(a[3][0] ** 2 + b[3][0] ** 2, rel=1e-14)
    assert ab[2][0] ** 2 == pytest.approx(a[2][0] ** 2 + b[2][0] ** 2, rel=1e-14)
    assert ab[0][0] == pytest.approx(a[0][0] * b[0][0], rel=1e-14)
    assert ab[1][0] == pytest.approx(a[1][0] + b[1][0], rel=1e-14)


def test_drift_reproduces_the_event_generator_widths():
    """The configs' depositions were drifted by the input generator with the
    same constants: the oracle's drift of the same points agrees (to the
    float32 rounding of the parameters)."""
    rng = np.random.default_rng(5)
    pts = np.stack([rng.uniform(0, 3600, 500), rng.uniform(0, 3000, 500), rng.uniform(0, 2400, 500)], 1)
    for kind, row in (("U", 0), ("V", 1), ("W", 2)):
        d = inputs._to_depos(pts, np.full(500, 1000.0), kind)
        params = (inputs.V_DRIFT, inputs.D_L, inputs.D_T, 0.0)
        q, t, st, sx, x = oracle.drift(params, d.q, np.zeros(500), pts[:, 0], pts[:, 1], pts[:, 2], PROJ)
        np.testing.assert_allclose(t, d.t, rtol=1e-6)
        np.testing.assert_allclose(st, d.sigma_t, rtol=1e-6)
        np.testing.assert_allclose(sx, d.sigma_x, rtol=1e-6)
        np.testing.assert_allclose(x[row], d.x, rtol=1e-6, atol=1e-3)
        np.testing.assert_array_equal(q, d.q.astype(np.float64))


@pytest.mark.parametrize("tau", [3000.0, 0.0])
def test_drift_adjoint_vs_central_differences(tau):
    n = 40
    q0, t0, xd, y, z = (a.astype(np.float64) for a in _groups(n, seed=8))
    xd[:3] = [0.0, -5.0, 1e-3]
    p64 = np.array([inputs.V_DRIFT, inputs.D_L, inputs.D_T, tau])
    rng = np.random.default_rng(2)
    gq, gt, gst, gsx = (rng.standard_normal(n) for _ in range(4))
    gx = rng.standard_normal((3, n))

    def dL(par_p, arrs_p, par_m, arrs_m):
        """L(+) - L(-) from the output differences (no cancellation against
        the large unperturbed part of L)."""
        op = stages.drift_f64(par_p, *arrs_p, PROJ)
        om = stages.drift_f64(par_m, *arrs_m, PROJ)
        return sum(np.sum(g * (a - b)) for g, a, b in zip((gq, gt, gst, gsx, gx), op, om))

    arrs = [q0, t0, xd, y, z]
    g = stages.drift_adjoint_f64(p64, *arrs, PROJ, gq, gt, gst, gsx, gx)
    for k in range(4):
        if tau == 0.0 and k == 3:
            assert g[5][3] == 0.0
            continue
        h = 1e-6 * abs(p64[k])
        pp, pm = p64.copy(), p64.copy()
        pp[k] += h
        pm[k] -= h
        fd = dL(pp, arrs, pm, arrs) / (2 * h)
        assert g[5][k] == pytest.approx(fd, rel=1e-6), k
    for a in range(5):
        for i in range(3, n, 4):
            h = 1e-6 * max(abs(arrs[a][i]), 1.0)
            ap = [x.copy() for x in arrs]
            am = [x.copy() for x in arrs]
            ap[a][i] += h
            am[a][i] -= h
            fd = dL(p64, ap, p64, am) / (2 * h)
            assert g[a][i] == pytest.approx(fd, rel=1e-6, abs=1e-8), (a, i)


# ------------------------------------------------------------------ noise

def _nplane(n_wires=64, n_ticks=1000, nt_fft=1024):
    return inputs.Plane(n_wires=n_wires, n_ticks=n_ticks, n_imp=1, nt_fft=nt_fft, nw_fft=n_wires, half_w=0)


def test_noise_normals_are_standard_and_independent():
    re, im = oracle.noise_normals(7, 1, 2, 200, 513)
    for a in (re.ravel(), im.ravel()):
        assert stats.kstest(a, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(re.ravel(), im.ravel())[0, 1]) < 0.015
    r2 = (re ** 2 + im ** 2).ravel()
    assert stats.kstest(r2, stats.chi2(2).cdf).pvalue > 1e-4
    # neighbouring wires / bins are uncorrelated
    assert abs(np.corrcoef(re[:-1].ravel(), re[1:].ravel())[0, 1]) < 0.015


def test_noise_counter_domain():
    """Normal pair of (wire, f) = Box-Muller of the Philox block with counter
    (wire, event, f, plane*2^24 + 2^23) under key = seed."""
    seed, ev, pl = 0xDEADBEEF12345678, 4, 2
    re, im = oracle.noise_normals(seed, ev, pl, 3, 5)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for w in range(3):
        for f in range(5):
            o = oracle.philox([w, ev, f, (pl << 24) + (1 << 23)], key)
            u1 = (int(o[0] >> 6) * 2 ** 26 + int(o[1] >> 6) + 0.5) * 2.0 ** -52
            u2 = (int(o[2] >> 6) * 2 ** 26 + int(o[3] >> 6) + 0.5) * 2.0 ** -52
            c, s = oracle.box_muller(u1, u2)
            assert (re[w, f], im[w, f]) == (c, s)


def test_noise_single_frequency_is_a_cosine():
    """With one non-zero amplitude A at bin f0 the waveform is
    (2/Tf) A (g_re cos(2 pi f0 t/Tf) - g_im sin(2 pi f0 t/Tf)); at the DC
    and Nyquist bins the real part alone, (1/Tf) A g_re (+-1)^t."""
    P = _nplane(n_wires=4)
    F, Tf = P.nt_fft // 2 + 1, P.nt_fft
    t = np.arange(P.n_ticks)
    for f0 in (0, 3, 100, F - 1):
        amp = np.zeros(F, np.float32)
        amp[f0] = 2.5
        N = oracle.noise(P, amp, 5, 0, 1)
        re, im = oracle.noise_normals(5, 0, 1, P.n_wires, F)
        for w in range(P.n_wires):
            if f0 in (0, F - 1):
                want = 2.5 * re[w, f0] * (-1.0) ** (t * (f0 == F - 1)) / Tf
            else:
                ang = 2 * np.pi * f0 * t / Tf
                want = 2 * 2.5 * (re[w, f0] * np.cos(ang) - im[w, f0] * np.sin(ang)) / Tf
            np.testing.assert_allclose(N[w], want, rtol=0, atol=1e-15)


def test_noise_variance_parseval():
    """Var N(t) = (A_0^2 + A_Nyq^2 + 4 sum_{0<f<Tf/2} A_f^2) / Tf^2 at every tick,
    and the mean power spectrum of full-length rows is 2 A_f^2."""
    P = _nplane(n_wires=3000, n_ticks=512, nt_fft=512)
    F, Tf = P.nt_fft // 2 + 1, P.nt_fft
    f = np.arange(F)
    amp = (1.0 + 0.01 * f + 3.0 * np.exp(-((f - 60) / 10.0) ** 2)).astype(np.float32)
    a = amp.astype(np.float64)
    N = oracle.noise(P, amp, 99, 2, 0)
    var_ref = (a[0] ** 2 + a[-1] ** 2 + 4 * np.sum(a[1:-1] ** 2)) / Tf ** 2
    assert N.var(axis=0).mean() == pytest.approx(var_ref, rel=0.01)
    psd = np.mean(np.abs(np.fft.rfft(N, axis=1)) ** 2, axis=0)
    ratio = psd[1:-1] / (2 * a[1:-1] ** 2)
    assert abs(ratio.mean() - 1) < 0.01 and np.all(np.abs(ratio - 1) < 6 * math.sqrt(1 / P.n_wires) + 0.05)


# ------------------------------------------------------------------ digitisation

def _f32_round(x: Fraction) -> Fraction:
    """Round an exact rational to the nearest float32 (ties to even), by hand."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = 0
    while a >= 2:
        a /= 2
        e += 1
    while a < 1:
        a *= 2
        e -= 1
    m = a * 2 ** 23
    fl = math.floor(m)
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * Fraction(fl) / 2 ** 23 * Fraction(2) ** e


def _rint_even(x: Fraction) -> int:
    fl = math.floor(x)
    rem = x - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


def test_digitize_hand_cases():
    v = np.array([2.5, 3.5, -3.0, 7e4, 1.4999999, 0.5, 4095.5, 4094.5], np.float32)
    got = oracle.digitize(v, 1.0, 0.0, 12)
    assert list(got) == [2, 4, 0, 4095, 1, 0, 4095, 4094]


def test_digitize_float32_operations_exact_rationals():
    """gain*v then + baseline, each rounded to float32, then rint (ties to
    even) and clipping, checked against exact rational arithmetic."""
    rng = np.random.default_rng(4)
    v = np.concatenate([rng.uniform(-300, 3000, 3000), rng.integers(-50, 2000, 500) + 0.5]).astype(np.float32)
    gain, base = np.float32(1.37), np.float32(900.25)
    got = oracle.digitize(v, gain, base, 12)
    for vi, gi in zip(v, got):
        y = _f32_round(_f32_round(Fraction(float(gain)) * Fraction(float(vi))) + Fraction(float(base)))
        assert gi == min(max(_rint_even(y), 0), 4095)
