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
//  k_wire_static the same with the plan fixed at compile time (Wf = 512:
//               8 8 8; Wf = 864: 6 4 6 6): first and last pass in
//               registers, one barrier per pass but the last;
//               k_wire_adjoint_static and k_wire_adjoint_offsets_static
//               (batched) likewise for the adjoint.
//  k_c2r_rows   inverse real FFT along ticks, scaled by 1/(Wf Tf), cropped.
//
// All three are bound by HBM traffic: every transform lives in LDS and each
// grid element is read and written once per pass.
#include <map>
#include <type_traits>
#include <mutex>
#include <utility>

#include "lar_internal.hpp"

namespace lar {

bool make_plan(int n, FftPlan* plan, int order) {
    if (n < 1 || order < 0 || order >= kPlanOrders) return false;
    int m = n, a = 0, b = 0;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    if (m != 1) return false;
    int r[kMaxPasses + 8], np = 0;
    auto twos_8 = [&]() {            // 2^a as 8s then one 4 or 2
        int x = a;
        while (x >= 3) { r[np++] = 8; x -= 3; }
        if (x == 2) r[np++] = 4;
        if (x == 1) r[np++] = 2;
    };
    auto threes = [&]() { for (int i = 0; i < b; ++i) r[np++] = 3; };
    if (order == 0 || order == 3) {
        twos_8();
        threes();
    } else if (order == 4) {
        int x = a, y = b;
        while (x >= 3) { r[np++] = 8; x -= 3; }
        while (x > 0 && y > 0) { r[np++] = 6; --x; --y; }
        if (x == 2) r[np++] = 4;
        if (x == 1) r[np++] = 2;
        for (int i = 0; i < y; ++i) r[np++] = 3;
    } else if (order == 5) {
        // radix 6 first and last; between them 8s, then a 4 or 2, then the
        // remaining 2 x 3 pairs as 6s, then 3s (864: 6 4 6 6)
        if (a < 2 || b < 2) return false;
        int x = a - 2, y = b - 2;
        r[np++] = 6;
        while (x >= 3 && x - 3 >= y) { r[np++] = 8; x -= 3; }
        while (x > y) {
            if (x - y >= 2) { r[np++] = 4; x -= 2; }
            else { r[np++] = 2; --x; }
        }
        while (x > 0 && y > 0) { r[np++] = 6; --x; --y; }
        for (int i = 0; i < y; ++i) r[np++] = 3;
        r[np++] = 6;
    } else if (order == 1) {
        int x = a;
        while (x >= 2) { r[np++] = 4; x -= 2; }
        threes();
        if (x == 1) r[np++] = 2;
    } else {
        threes();
        twos_8();
    }
    if (np > kMaxPasses) return false;
    for (int i = 0; i < np; ++i) plan->radix[i] = order == 3 ? r[np - 1 - i] : r[i];
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


// Half-angle table h[k] = exp(-pi i k / Nh) = exp(-2 pi i k / Tf), k < Nh,
// computed in double and rounded once.  When 4 divides Nh, only the first
// octant's angles (k <= Nh/4) are evaluated and the other three quarters
// of the table are their reflections (cos and sin swapped or negated): a
// quarter of the double-precision sincospi calls, which each workgroup
// makes before its first row.  Every entry is written by one thread.
__device__ __forceinline__ void fill_half_table(float2* h, int Nh, int tid, int T) {
    if ((Nh & 3) == 0) {
        const int Q = Nh >> 2, H = Nh >> 1;
        for (int i = tid; i <= Q; i += T) {
            double s, c;
            sincospi((double)i / (double)Nh, &s, &c);
            const float fc = (float)c, fs = (float)s;
            h[i] = make_float2(fc, -fs);                           // angle t
            if (i >= 1 && i < Q) h[H - i] = make_float2(fs, -fc);  // pi/2 - t
            if (i < Q) h[H + i] = make_float2(-fs, -fc);           // pi/2 + t
            if (i >= 1) h[Nh - i] = make_float2(-fc, -fs);         // pi - t
        }
        return;
    }
    for (int i = tid; i < Nh; i += T) {
        double s, c;
        sincospi(-(double)i / (double)Nh, &s, &c);
        h[i] = make_float2((float)c, (float)s);
    }
}

// Even/odd sample pairs of one row into registers, pair n = tid + i*T, in
// two halves: issue_row_pairs only issues the loads (unconditional, with
// addresses clamped into the row), and row_pair masks a loaded pair when it
// is stored to LDS.  Nothing reads the loaded registers in between, so the
// next row's loads stay in flight across the current row's transform (a
// select right after the loads would make the compiler wait for them before
// the transform).  pairs_ok (n_in even, 8-byte aligned rows): one 8-byte
// load per pair; else two 4-byte loads.
template <int VPT>
__device__ __forceinline__ void issue_row_pairs(const float* __restrict__ x, int n_in, int tid, int T,
                                                bool pairs_ok, float2 (&raw)[VPT]) {
    if (pairs_ok) {
        const float2* x2 = reinterpret_cast<const float2*>(x);
        const int last = (n_in >> 1) - 1;
#pragma unroll
        for (int i = 0; i < VPT; ++i) raw[i] = x2[min(tid + i * T, last)];
    } else {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int n = tid + i * T;
            raw[i] = make_float2(x[min(2 * n, n_in - 1)], x[min(2 * n + 1, n_in - 1)]);
        }
    }
}

__device__ __forceinline__ float2 row_pair(float2 raw, int n, int n_in) {
    return make_float2(2 * n < n_in ? raw.x : 0.f, 2 * n + 1 < n_in ? raw.y : 0.f);
}

// LDS of the row kernels: the padded transform buffer, the half-angle
// table h and, with PM, the pass-major twiddle tables.
static size_t row_lds_bytes(const FftPlan& plan, bool pm) {
    return ((size_t)lds_slots(plan.n, 1) + plan.n + (pm ? pm_entries(plan) : 0)) * sizeof(float2);
}

// Row transform with the twiddles of the half table (TwHalf) or of the
// pass-major tables (PM); p0 = 1 when the first pass ran in registers.
template <int VPT, int PM>
__device__ __forceinline__ void row_fft(float2* A, const FftPlan& plan, int tid, int T, const float2* h,
                                        const float2* tp, bool inv, int p0) {
    if (PM) {
        fft_lds_pm<VPT, 1, 1>(A, plan, tid, T, tp, inv, p0);
    } else {
        // (p0 is 0 here: the register first pass is used with PM only)
        const TwHalf tw{h, plan.n};
        int Ns = 1;
        for (int p = 0; p < plan.npass; ++p) {
            const int R = plan.radix[p];
            if (R == 8) stockham_pass_tw<8, (VPT + 7) / 8>(A, plan.n, Ns, tid, T, tw, inv);
            else if (R == 6) stockham_pass_tw<6, (VPT + 5) / 6>(A, plan.n, Ns, tid, T, tw, inv);
            else if (R == 4) stockham_pass_tw<4, (VPT + 3) / 4>(A, plan.n, Ns, tid, T, tw, inv);
            else if (R == 3) stockham_pass_tw<3, (VPT + 2) / 3>(A, plan.n, Ns, tid, T, tw, inv);
            else stockham_pass_tw<2, (VPT + 1) / 2>(A, plan.n, Ns, tid, T, tw, inv);
            Ns *= R;
        }
    }
}

// Split step of the real FFT from the Tf/2-point complex transform Z in A:
// X[k] = (Z[k] + Z*[Nh-k])/2 - i W^k (Z[k] - Z*[Nh-k])/2, W = exp(-2 pi i / Tf),
// written for k <= Nh/2 and Nh - k.
__device__ __forceinline__ void r2c_split(const float2* A, const float2* h, int Nh, int tid, int T,
                                          float2* __restrict__ y) {
    for (int k = tid; k <= Nh / 2; k += T) {
        float2 zk = A[lidx<1>(k)], zm = A[lidx<1>(k == 0 ? 0 : Nh - k)];
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

// Time-axis real FFT of rows: Tf real samples (n_in read, the rest zero)
// as a Tf/2-point complex FFT of even/odd pairs, then the split step.  A
// persistent workgroup loops over rows and loads the next row while the
// current one is transformed.  When every thread holds exactly the inputs
// of one first-pass butterfly (VPT = first radix, NT * VPT = Tf/2) that
// pass runs in registers straight from the loads.  SF (optional): the
// remaining passes with the plan fixed at compile time (InplaceRowFft).
template <int VPT, int NT, int PM, int REG, class SF = void>
__global__ __launch_bounds__(NT) void k_r2c_rows(const float* __restrict__ in,
                                                          int64_t ld_in, int n_in, int nrows,
                                                          FftPlan plan, float2* __restrict__ out,
                                                          int64_t ld_out, int pairs_ok,
                                                          const int64_t* __restrict__ row_in) {
    extern __shared__ float2 lds[];
    const int Nh = plan.n, tid = threadIdx.x, T = NT;
    float2* A = lds;
    float2* h = lds + lds_slots(Nh, 1);
    float2* tp = h + Nh;
    fill_half_table(h, Nh, tid, T);
    if (PM) {
        lds_barrier();
        build_pm(tp, plan, TwHalf{h, Nh}, tid, T);
    }
    // REG (chosen by the launcher): plan.radix[0] == VPT, NT * VPT == Nh,
    // and rows of even length at 8-byte aligned starts (pairs_ok)
    constexpr bool kReg = REG && (VPT == 2 || VPT == 4 || VPT == 8);
    float2 v[VPT];
    // input row r starts at row_in[r] when given, else at r * ld_in
    auto row_ptr = [&](int r) { return in + (row_in ? row_in[r] : (int64_t)r * ld_in); };
    int row = blockIdx.x;
    if constexpr (kReg) {
        // lean loop: one 8-byte load per pair, the pair masked as a whole
        const int last = (n_in >> 1) - 1;
        auto issue = [&](int r) {
            const float2* x2 = reinterpret_cast<const float2*>(row_ptr(r));
#pragma unroll
            for (int i = 0; i < VPT; ++i) v[i] = x2[min(tid + i * T, last)];
        };
        if (row < nrows) issue(row);
        for (; row < nrows; row += gridDim.x) {
            lds_barrier();
            // thread tid holds z[tid + r T], the inputs of butterfly tid of the
            // first pass (Ns = 1: no twiddles); its outputs go to tid * VPT + r
            float2 u[VPT];
#pragma unroll
            for (int i = 0; i < VPT; ++i) u[i] = 2 * (tid + i * T) < n_in ? v[i] : make_float2(0.f, 0.f);
            if (row + (int)gridDim.x < nrows) issue(row + gridDim.x);
            dft_small<VPT>(u, false);
#pragma unroll
            for (int r = 0; r < VPT; ++r) A[lidx<1>(tid * VPT + r)] = u[r];
            lds_barrier();
            if constexpr (std::is_void<SF>::value) row_fft<VPT, PM>(A, plan, tid, T, h, tp, false, 1);
            else SF::run(A, tp, tid, false);   // the passes after the first, compile-time plan
            r2c_split(A, h, Nh, tid, T, out + (int64_t)row * ld_out);
        }
        return;
    }
    if (row < nrows) issue_row_pairs<VPT>(row_ptr(row), n_in, tid, T, pairs_ok != 0, v);
    for (; row < nrows; row += gridDim.x) {
        lds_barrier();
        {
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                int n = tid + i * T;
                if (n < Nh) A[lidx<1>(n)] = row_pair(v[i], n, n_in);
            }
            // prefetch the next row of this workgroup while this one is transformed
            if (row + (int)gridDim.x < nrows)
                issue_row_pairs<VPT>(row_ptr(row + gridDim.x), n_in, tid, T, pairs_ok != 0, v);
            lds_barrier();
            row_fft<VPT, PM>(A, plan, tid, T, h, tp, false, 0);
        }
        r2c_split(A, h, Nh, tid, T, out + (int64_t)row * ld_out);
    }
}

// Bins k = tid + i*T (k <= Nh/2) and Nh - k of one spectrum row into registers.
template <int VPT>
__device__ __forceinline__ void load_spec_pairs(const float2* __restrict__ X, int Nh, int tid, int T,
                                                float2 (&a)[VPT], float2 (&b)[VPT]) {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        int k = min(tid + i * T, Nh / 2);
        a[i] = X[k];
        b[i] = X[Nh - k];
    }
}

template <int VPT, int NT, int PM, class SF = void>
__global__ __launch_bounds__(NT) void k_c2r_rows(const float2* __restrict__ in,
                                                          int64_t ld_in, int nrows, FftPlan plan,
                                                          float* __restrict__ out, int64_t ld_out,
                                                          int n_out, float scale, int pairs_ok,
                                                          const int64_t* __restrict__ row_off) {
    extern __shared__ float2 lds[];
    const int Nh = plan.n, tid = threadIdx.x, T = NT;
    float2* A = lds;
    float2* h = lds + lds_slots(Nh, 1);
    float2* tp = h + Nh;
    fill_half_table(h, Nh, tid, T);
    if (PM) {
        lds_barrier();
        build_pm(tp, plan, TwHalf{h, Nh}, tid, T);
    }
    // the pre-step touches Nh/2 + 1 bin pairs: VPT/2 (rounded up) per thread
    constexpr int VH = (VPT + 1) / 2 + 1;
    float2 xa[VH], xb[VH];
    int row = blockIdx.x;
    if (row < nrows) load_spec_pairs<VH>(in + (int64_t)row * ld_in, Nh, tid, T, xa, xb);
    for (; row < nrows; row += gridDim.x) {
        lds_barrier();
        // pre-step: Z[k] = (X[k] + X*[Nh-k]) + i (X[k] - X*[Nh-k]) exp(+2 pi i k/Tf),
        // the imaginary parts of the DC and Nyquist bins are dropped
#pragma unroll
        for (int i = 0; i < VH; ++i) {
            int k = tid + i * T;
            if (k <= Nh / 2) {
                float2 xk = xa[i], xm = xb[i];
                if (k == 0) { xk.y = 0.f; xm.y = 0.f; }
                float2 w = h[k];
                float2 a1 = make_float2(xk.x + xm.x, xk.y - xm.y);
                float2 b1 = cmulc(make_float2(xk.x - xm.x, xk.y + xm.y), w);   // * exp(+2 pi i k/Tf)
                float2 a2 = make_float2(xm.x + xk.x, xm.y - xk.y);
                float2 b2 = cmul(make_float2(xm.x - xk.x, xm.y + xk.y), make_float2(-w.x, -w.y));
                A[lidx<1>(k)] = make_float2(a1.x - b1.y, a1.y + b1.x);
                if (k > 0) A[lidx<1>(Nh - k)] = make_float2(a2.x - b2.y, a2.y + b2.x);
            }
        }
        if (row + (int)gridDim.x < nrows)
            load_spec_pairs<VH>(in + (int64_t)(row + gridDim.x) * ld_in, Nh, tid, T, xa, xb);
        lds_barrier();
        if constexpr (std::is_void<SF>::value) row_fft<VPT, PM>(A, plan, tid, T, h, tp, true, 0);
        else SF::run(A, tp, tid, true);   // compile-time plan
        float* y = out + (row_off ? row_off[row] : (int64_t)row * ld_out);
        if (pairs_ok) {
            float2* y2 = reinterpret_cast<float2*>(y);
            const int full = n_out >> 1;
            for (int n = tid; n < Nh; n += T) {
                float2 z = A[lidx<1>(n)];
                if (n < full) y2[n] = make_float2(z.x * scale, z.y * scale);
                else if (2 * n < n_out) y[2 * n] = z.x * scale;
            }
        } else {
            for (int n = tid; n < Nh; n += T) {
                float2 z = A[lidx<1>(n)];
                if (2 * n < n_out) y[2 * n] = z.x * scale;
                if (2 * n + 1 < n_out) y[2 * n + 1] = z.y * scale;
            }
        }
    }
}

// Per-kernel launch facts cached on the host: the dynamic LDS limit set so
// far and the resident workgroups per CU for a (threads, LDS) launch, so
// that a launch makes no attribute or occupancy query once they are known.
namespace {
struct KernelFacts {
    size_t lds_set = 65536;                  // larger sizes need the attribute
    std::map<std::pair<int, size_t>, int> per_cu;
};
std::mutex g_facts_mu;
std::map<std::pair<int, const void*>, KernelFacts> g_facts;   // (device, kernel)

KernelFacts& facts(const void* k) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return g_facts[std::make_pair(dev, k)];
}
}  // namespace

template <class K>
static void set_lds(K kernel, size_t bytes) {
    const void* k = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(g_facts_mu);
    KernelFacts& f = facts(k);
    if (bytes > f.lds_set &&
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        f.lds_set = bytes;
}

template <class K>
static int blocks_per_cu(K kernel, int threads, size_t lds) {
    const void* k = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(g_facts_mu);
    KernelFacts& f = facts(k);
    const auto key = std::make_pair(threads, lds);
    auto it = f.per_cu.find(key);
    if (it != f.per_cu.end()) return it->second;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, threads, lds) != hipSuccess || per < 1) per = 1;
    f.per_cu[key] = per;
    return per;
}

// Persistent grid of a row kernel: as many workgroups as are resident at
// once (occupancy from the kernel's registers and this launch's LDS), at
// most one per row.
template <class K>
static int row_grid(K kernel, int threads, size_t lds, int nrows) {
    const int g = blocks_per_cu(kernel, threads, lds) * device_cus();
    return nrows < g ? nrows : g;
}

// The pass-major tables fit next to the buffer and the half table.
static bool row_pm(const FftPlan& plan) { return row_lds_bytes(plan, true) <= kLdsBytes; }

// Values per thread of a transform of n points over T threads, rounded up to
// the instantiated 1, 2, 4 or 8; 0 if more than 8 would be needed.
static int vpt_for(int n, int T) {
    const int need = (n + T - 1) / T;
    for (int v = 1; v <= 8; v *= 2)
        if (need <= v) return v;
    return 0;
}

// Rows: Nh/8 threads when that is a listed size (each thread then holds the
// 8 inputs of one first-pass butterfly and that pass runs in registers;
// measured fastest at Tf = 6144), else 256 / 512 / 1024 by length.
int default_row_threads(int nt_fft) {
    const int Nh = nt_fft / 2;
    if (Nh % 8 == 0) {
        const int t = Nh / 8;
        if (t == 256 || t == 384 || t == 512 || t == 768 || t == 1024) return t;
    }
    return Nh <= 1024 ? 256 : Nh <= 4096 ? 512 : 1024;
}

bool row_sched_ok(int nt_fft, int threads, int order) {
    FftPlan plan;
    return (threads == 256 || threads == 384 || threads == 512 || threads == 768 || threads == 1024) &&
           vpt_for(nt_fft / 2, threads) &&
           make_plan(nt_fft / 2, &plan, order);
}

// Instantiations: T in {256, 384, 512, 768, 1024} threads by V in
// {1, 2, 4, 8} values per thread (384 and 768 hold the 3 * 2^k lengths
// exactly); f(V, T) is called with the pair that a schedule selects.
#define LAR_ROW_DISPATCH(V, T, X)                                   \
    switch ((T) * 16 + (V)) {                                       \
        case 256 * 16 + 1: X(1, 256) break;                         \
        case 256 * 16 + 2: X(2, 256) break;                         \
        case 256 * 16 + 4: X(4, 256) break;                         \
        case 256 * 16 + 8: X(8, 256) break;                         \
        case 384 * 16 + 1: X(1, 384) break;                         \
        case 384 * 16 + 2: X(2, 384) break;                         \
        case 384 * 16 + 4: X(4, 384) break;                         \
        case 384 * 16 + 8: X(8, 384) break;                         \
        case 768 * 16 + 1: X(1, 768) break;                         \
        case 768 * 16 + 2: X(2, 768) break;                         \
        case 768 * 16 + 4: X(4, 768) break;                         \
        case 768 * 16 + 8: X(8, 768) break;                         \
        case 512 * 16 + 1: X(1, 512) break;                         \
        case 512 * 16 + 2: X(2, 512) break;                         \
        case 512 * 16 + 4: X(4, 512) break;                         \
        case 512 * 16 + 8: X(8, 512) break;                         \
        case 1024 * 16 + 1: X(1, 1024) break;                       \
        case 1024 * 16 + 2: X(2, 1024) break;                       \
        case 1024 * 16 + 4: X(4, 1024) break;                       \
        case 1024 * 16 + 8: X(8, 1024) break;                       \
        default: return hipErrorInvalidValue;                       \
    }

// Row kernels: one row per workgroup at a time, a persistent grid of
// 4 workgroups per CU.  threads = 0 selects the default: 256 threads for
// half-lengths up to 1024, 512 up to 4096 and 1024 above.
// Tf/2 = 3072 with the plan 8 8 8 6 (radix order 4) has compile-time row kernels.
static bool plan_is_8886(const FftPlan& plan) {
    return plan.n == 3072 && plan.npass == 4 && plan.radix[0] == 8 && plan.radix[1] == 8 && plan.radix[2] == 8 &&
           plan.radix[3] == 6;
}

hipError_t launch_r2c_rows(const float* in, int64_t ld_in, int n_in, int nrows, int nt_fft,
                           float2* out, int64_t ld_out, hipStream_t s, int threads, int order,
                           const int64_t* row_in, bool row_in_even) {
    if (!threads) threads = default_row_threads(nt_fft);
    FftPlan plan;
    if (!make_plan(nt_fft / 2, &plan, order)) return hipErrorInvalidValue;
    const int Nh = plan.n, vpt = vpt_for(Nh, threads);
    if (!vpt) return hipErrorInvalidValue;
    if (nrows <= 0) return hipSuccess;
    const bool pm = row_pm(plan);
    const size_t lds = row_lds_bytes(plan, pm);
    const int pairs_ok = ((ld_in % 2) == 0 && (n_in % 2) == 0 && (reinterpret_cast<uintptr_t>(in) % 8) == 0 &&
                          (row_in == nullptr || row_in_even))
                             ? 1
                             : 0;
    // the first pass runs in registers when each thread holds one butterfly
    const bool reg = pm && pairs_ok && plan.radix[0] == vpt && threads * vpt == Nh && vpt >= 2;
    if (reg && threads == 384 && plan_is_8886(plan)) {   // Tf = 6144 with the default plan
        using SF = InplaceRowFft<3072, 384, 8, 7, 8, 8, 6>;
        auto kern = k_r2c_rows<8, 384, 1, 1, SF>;
        set_lds(kern, lds);
        hipLaunchKernelGGL(kern, dim3(row_grid(kern, 384, lds, nrows)), dim3(384), lds, s, in, ld_in, n_in, nrows,
                           plan, out, ld_out, pairs_ok, row_in);
        return hipGetLastError();
    }
#define LAR_R2C_PM(V, T, PM, RG)                                                                      \
    {                                                                                                 \
        set_lds(k_r2c_rows<V, T, PM, RG>, lds);                                                       \
        dim3 grid(row_grid(k_r2c_rows<V, T, PM, RG>, T, lds, nrows));                                 \
        hipLaunchKernelGGL((k_r2c_rows<V, T, PM, RG>), grid, dim3(T), lds, s, in, ld_in, n_in, nrows,  \
                           plan, out, ld_out, pairs_ok, row_in);                                      \
    }
#define LAR_R2C(V, T)                   \
    if (reg) LAR_R2C_PM(V, T, 1, 1)     \
    else if (pm) LAR_R2C_PM(V, T, 1, 0) \
    else LAR_R2C_PM(V, T, 0, 0)
    LAR_ROW_DISPATCH(vpt, threads, LAR_R2C)
#undef LAR_R2C
#undef LAR_R2C_PM
    return hipGetLastError();
}

hipError_t launch_c2r_rows(const float2* in, int64_t ld_in, int nrows, int nt_fft, float* out,
                           int64_t ld_out, int n_out, float scale, hipStream_t s,
                           const int64_t* row_off, bool row_off_even, int threads, int order) {
    if (!threads) threads = default_row_threads(nt_fft);
    FftPlan plan;
    if (!make_plan(nt_fft / 2, &plan, order)) return hipErrorInvalidValue;
    const int Nh = plan.n, vpt = vpt_for(Nh, threads);
    if (!vpt) return hipErrorInvalidValue;
    if (nrows <= 0) return hipSuccess;
    const bool pm = row_pm(plan);
    const size_t lds = row_lds_bytes(plan, pm);
    const int pairs_ok = ((ld_out % 2) == 0 && (reinterpret_cast<uintptr_t>(out) % 8) == 0 &&
                          (row_off == nullptr || row_off_even))
                             ? 1
                             : 0;
    if (pm && threads == 384 && plan_is_8886(plan)) {   // Tf = 6144 with the default plan
        using SF = InplaceRowFft<3072, 384, 1, 0, 8, 8, 8, 6>;
        auto kern = k_c2r_rows<8, 384, 1, SF>;
        set_lds(kern, lds);
        hipLaunchKernelGGL(kern, dim3(row_grid(kern, 384, lds, nrows)), dim3(384), lds, s, in, ld_in, nrows, plan,
                           out, ld_out, n_out, scale, pairs_ok, row_off);
        return hipGetLastError();
    }
#define LAR_C2R_PM(V, T, PM)                                                                    \
    {                                                                                           \
        set_lds(k_c2r_rows<V, T, PM>, lds);                                                     \
        dim3 grid(row_grid(k_c2r_rows<V, T, PM>, T, lds, nrows));                               \
        hipLaunchKernelGGL((k_c2r_rows<V, T, PM>), grid, dim3(T), lds, s, in, ld_in, nrows, plan, \
                           out, ld_out, n_out, scale, pairs_ok, row_off);                       \
    }
#define LAR_C2R(V, T)               \
    if (pm) LAR_C2R_PM(V, T, 1)     \
    else LAR_C2R_PM(V, T, 0)
    LAR_ROW_DISPATCH(vpt, threads, LAR_C2R)
#undef LAR_C2R
#undef LAR_C2R_PM
    return hipGetLastError();
}

// ---------------------------------------------------------------- wire pass


__device__ __forceinline__ void fill_full_table(float2* t, int n, int tid, int T) {
    for (int i = tid; i < n; i += T) {
        double s, c;
        sincospi(-2.0 * (double)i / (double)n, &s, &c);
        t[i] = make_float2((float)c, (float)s);
    }
}

// Pass-major twiddle tables of an n-point plan straight from FP64 sincospi
// (rounded once), for kernels without a full table in LDS.
__device__ __forceinline__ void build_pm_direct(float2* tp, const FftPlan& plan, int tid, int T) {
    int Ns = 1, off = 0;
    for (int p = 0; p < plan.npass; ++p) {
        const int R = plan.radix[p], cnt = Ns * (R - 1), stride = plan.n / (Ns * R);
        for (int e = tid; e < cnt; e += T) {
            const int k = e / (R - 1), r = e - k * (R - 1) + 1;
            double sn, cs;
            sincospi(-2.0 * (double)(r * k * stride) / (double)plan.n, &sn, &cs);
            tp[off + e] = make_float2((float)cs, (float)sn);
        }
        off += cnt;
        Ns *= R;
    }
}

// LDS of the wire pass: the padded [Wf][C] tile and the pass-major tables.
static size_t wire_lds_bytes(const FftPlan& plan, int C) {
    return ((size_t)lds_slots(plan.n * C, 1) + pm_entries(plan)) * sizeof(float2);
}

// First step of the transform of the [Wf][C] tile whose element
// e = tid + i T the thread holds in x[i] (wire p = e / C, column e % C):
// x goes to LDS, or, with REG (x holds the inputs of the thread's
// first-pass butterfly: VPT = first radix, T / C = Wf / VPT), that pass runs
// in registers and its outputs go to LDS.  x is dead afterwards; wire_fft_rest
// finishes the transform in A.
template <int VPT, int C, int REG>
__device__ __forceinline__ void wire_fft_first(float2* A, int tid, int T, float2 (&x)[VPT], int nel, bool inv) {
    if constexpr (REG != 0 && (VPT == 2 || VPT == 4 || VPT == 8)) {
        dft_small<VPT>(x, inv);
        const int j = tid / C, sc = tid % C;
#pragma unroll
        for (int r = 0; r < VPT; ++r) A[lidx<1>((j * VPT + r) * C + sc)] = x[r];
    } else {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + i * T;
            if (e < nel) A[lidx<1>(e)] = x[i];
        }
    }
}
template <int VPT, int C, int REG, bool R6>
__device__ __forceinline__ void wire_fft_rest(float2* A, const FftPlan& plan, int tid, int T, const float2* tp,
                                              bool inv) {
    lds_barrier();
    constexpr int p0 = (REG != 0 && (VPT == 2 || VPT == 4 || VPT == 8)) ? 1 : 0;
    fft_lds_pm<VPT, C, 1, R6>(A, plan, tid, T, tp, inv, p0);
}

static bool plan_has6(const FftPlan& plan) {
    for (int p = 0; p < plan.npass; ++p)
        if (plan.radix[p] == 6) return true;
    return false;
}

// One workgroup per tile of C consecutive time-frequency columns.
template <int VPT, int C, int NT, int REG, bool R6>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_wire_fused(
    const float2* __restrict__ S, int64_t ldS, int n_wires, int n_imp, int F, FftPlan plan,
    const float2* __restrict__ R, float2* __restrict__ M, int64_t ldM, int64_t strideS,
    int64_t strideM, int batch) {
    extern __shared__ float2 lds[];
    // block -> (tile, item) of a batch sharing this plane shape and response
    int tile, item;
    tile_item(xcd_tile(blockIdx.x, gridDim.x), (F + C - 1) / C, batch, C, tile, item);
    S += (int64_t)item * strideS;
    M += (int64_t)item * strideM;
    const int Wf = plan.n, tid = threadIdx.x, T = NT;
    float2* A = lds;                                  // [Wf][C], padded
    float2* tp = lds + lds_slots(Wf * C, 1);          // pass-major twiddles
    build_pm_direct(tp, plan, tid, T);
    const int f0 = tile * C;
    const int nel = Wf * C;
    float2 acc[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) acc[i] = make_float2(0.f, 0.f);

    // element e = tid + i*T of the tile is (wire p = e / C, column c = e % C);
    // every gather below is unconditional (clamped address, value masked)
    // so that a thread's loads are all in flight together.  The next
    // offset's grid rows are requested before this offset's FFT and its
    // response slab right after this offset's product, so both loads
    // overlap an FFT.
    float2 v[VPT], r[VPT];
    // (T is a multiple of C, so a thread's column is fixed and its wire
    // advances by T / C per i.)  The row index passes through an empty asm
    // so that the per-i addresses are rebuilt for each gather rather than
    // hoisted out of the offset loop, where they would pin 2 VPT registers.
    static_assert(NT % C == 0, "tile width must divide the thread count");
    const int c_own = tid % C, p_own = tid / C, f_own = min(f0 + c_own, F - 1);
    const bool f_ok = f0 + c_own < F;
    // (the rows are loaded raw and masked only when they are used: a select
    // right after the loads would make the compiler wait for them before the
    // FFT they are meant to overlap)
    auto gather_s = [&](int k) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            int p = p_own + i * (NT / C);
            asm volatile("" : "+v"(p));
            v[i] = S[(int64_t)(min(p, n_wires - 1) * n_imp + k) * ldS + f_own];
        }
    };
    auto gather_r = [&](int k) {
        const float2* Rk = R + (int64_t)k * Wf * F;
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            int p = p_own + i * (NT / C);
            asm volatile("" : "+v"(p));
            r[i] = Rk[(int64_t)min(p, Wf - 1) * F + f_own];
        }
    };
    gather_s(0);
    gather_r(0);
    for (int k = 0; k < n_imp; ++k) {
        lds_barrier();
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const bool ok = f_ok && p_own + i * (NT / C) < n_wires;   // n_wires <= Wf
            v[i] = ok ? v[i] : make_float2(0.f, 0.f);
        }
        wire_fft_first<VPT, C, REG>(A, tid, T, v, nel, false);
        if (k + 1 < n_imp) gather_s(k + 1);
        wire_fft_rest<VPT, C, REG, R6>(A, plan, tid, T, tp, false);
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            int e = tid + i * T;
            if (e < nel) {
                float2 a = A[lidx<1>(e)];
                acc[i].x += a.x * r[i].x - a.y * r[i].y;
                acc[i].y += a.x * r[i].y + a.y * r[i].x;
            }
        }
        if (k + 1 < n_imp) gather_r(k + 1);
    }
    lds_barrier();
    wire_fft_first<VPT, C, REG>(A, tid, T, acc, nel, true);
    wire_fft_rest<VPT, C, REG, R6>(A, plan, tid, T, tp, true);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        int e = tid + i * T;
        if (e < nel) {
            int p = e / C, c = e % C, f = f0 + c;
            if (p < n_wires && f < F) M[(int64_t)p * ldM + f] = A[lidx<1>(e)];
        }
    }
}

// The wire pass with its plan fixed at compile time: radices R0, Rm..., R0
// (first and last radix equal) over N wires, one first- and last-pass
// butterfly per thread (T = C N / R0).  Thread (j, s) = (tid / C, tid % C)
// holds wires j + (N / R0) r, r < R0, of column s: exactly the inputs of its
// first-pass butterfly and the outputs of its last-pass one (a Stockham last
// pass writes butterfly j's outputs to j + r N / R0).  So per impact offset
// the gathered rows go through the first pass in registers, the middle
// passes between two LDS buffers (no barrier between a pass's reads and its
// writes), the last pass back into registers, where its outputs meet the
// response slab: one barrier per pass but the last, and every LDS index is
// a thread constant plus a compile-time offset.  The sum over offsets goes
// through the same passes inverted.
// One middle Stockham pass (radix R, sub-transform size NS) of C interleaved
// N-point transforms from src to dst (both padded).
template <int N, int C, int NT, int NS, int R>
__device__ __forceinline__ void static_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                                            const float2* __restrict__ tw, int tid, bool inv) {
    constexpr int NB = N / R, TOT = NB * C, MAXB = (TOT + NT - 1) / NT;
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int w = tid + m * NT;
        if (TOT % NT == 0 || w < TOT) {
            const int s = w % C, b = w / C, k = b % NS;
            const int ib = b * C + s, li = lidx<1>(ib);
            float2 x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // (when NB C is a multiple of 32 the pad advances by exactly NB C / 32)
                float2 y = src[(NB * C) % 32 == 0 ? li + r * (NB * C + NB * C / 32) : lidx<1>(ib + r * NB * C)];
                if (r > 0) y = inv ? cmulc(y, tw[k * (R - 1) + r - 1]) : cmul(y, tw[k * (R - 1) + r - 1]);
                x[r] = y;
            }
            dft_small<R>(x, inv);
            const int ob = ((b - k) * R + k) * C + s, lo = lidx<1>(ob);
#pragma unroll
            for (int r = 0; r < R; ++r)
                dst[(NS * C) % 32 == 0 ? lo + r * (NS * C + NS * C / 32) : lidx<1>(ob + r * NS * C)] = x[r];
        }
    }
}

template <int N, int C, int NT, int NS, int TOFF>
__device__ __forceinline__ void static_mid(RadixList<>, float2*&, float2*&, const float2*, int, bool) {}
template <int N, int C, int NT, int NS, int TOFF, int R, int... Rest>
__device__ __forceinline__ void static_mid(RadixList<R, Rest...>, float2*& src, float2*& dst, const float2* tp,
                                           int tid, bool inv) {
    static_pass<N, C, NT, NS, R>(src, dst, tp + TOFF, tid, inv);
    lds_barrier();
    float2* t = src;
    src = dst;
    dst = t;
    static_mid<N, C, NT, NS * R, TOFF + NS * (R - 1)>(RadixList<Rest...>{}, src, dst, tp, tid, inv);
}

// C interleaved N-point transforms over wires with the plan fixed at compile
// time, for a workgroup of NT = C N / R0 threads: thread (j, s) holds the
// values at j + (N / R0) r, r < R0, of column s on entry and on exit (the
// inputs of its first-pass butterfly, the outputs of its last-pass one).
// The LDS holds two padded [N][C] buffers and the pass-major twiddles.
template <int N, int C, int NT, int R0, int... Rm>
struct StaticFft {
    static constexpr int NB = N / R0;                      // wire stride of a thread's values
    static constexpr int SL = N * C + N * C / 32;          // padded slots of one buffer
    static constexpr int P = 2 + sizeof...(Rm);            // passes
    static constexpr int TL = R0 - 1 + TableSpan<R0, Rm...>::v;   // table entry of the last pass
    static_assert(NB * C == NT, "one first- and last-pass butterfly per thread");
    static_assert(R0 * RadixProd<Rm...>::v * R0 == N, "plan length");
    float2* buf0;
    float2* buf1;
    float2* tp;
    int tid, j, s, e0, i1, li1, par;
    // builds the twiddle table; the first barrier of run, before any pass
    // reads it, orders the build
    __device__ StaticFft(float2* lds, const FftPlan& plan, int tid_)
        : buf0(lds), buf1(lds + SL), tp(lds + 2 * SL), tid(tid_), j(tid_ / C), s(tid_ % C), par(0) {
        e0 = j * R0 * C + s;
        i1 = j * C + s;
        li1 = lidx<1>(i1);
        build_pm_direct(tp, plan, tid, NT);
    }
    static size_t lds_bytes(const FftPlan& plan) {
        return (size_t)(2 * SL + pm_entries(plan)) * sizeof(float2);
    }
    // x <- the (inverse with inv) transform of x.  With an even number of
    // passes the last pass reads the buffer the first pass writes, so
    // successive transforms start on alternate buffers: the first pass of
    // one then never overwrites what the last pass of the previous one may
    // still be reading.
    __device__ __forceinline__ void run(float2 (&x)[R0], bool inv) {
        float2* a = (P % 2 == 0 && par) ? buf1 : buf0;
        float2* b = (P % 2 == 0 && par) ? buf0 : buf1;
        par ^= 1;
        dft_small<R0>(x, inv);
#pragma unroll
        for (int r = 0; r < R0; ++r) a[lidx<1>(e0 + r * C)] = x[r];
        lds_barrier();
        static_mid<N, C, NT, R0, R0 - 1>(RadixList<Rm...>{}, a, b, tp, tid, inv);
        const float2* tl = tp + TL;   // a holds the last pass's inputs
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            float2 y = a[(NB * C) % 32 == 0 ? li1 + r * (NB * C + NB * C / 32) : lidx<1>(i1 + r * NB * C)];
            if (r > 0) y = inv ? cmulc(y, tl[j * (R0 - 1) + r - 1]) : cmul(y, tl[j * (R0 - 1) + r - 1]);
            x[r] = y;
        }
        dft_small<R0>(x, inv);
    }
};

// The wire pass with a compile-time plan: per impact offset the gathered
// rows go through the first pass in registers, the middle passes between
// two LDS buffers (no barrier between a pass's reads and its writes), and
// the last pass back into registers, where its outputs meet the response
// slab: one barrier per pass but the last, and every LDS index is a thread
// constant plus a compile-time offset.  The sum over offsets goes through
// the same passes inverted.  PREF: the next offset's response slab is
// requested right after this offset's product (else right after this
// offset's transform, which spares its registers: with 576 threads, two
// workgroups per CU need at most 96 per lane).
template <int N, int C, int NT, bool PREF, int R0, int... Rm>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 576 ? 5 : 4, 8)))
void k_wire_static(const float2* __restrict__ S, int64_t ldS, int n_wires, int n_imp, int F, FftPlan plan,
                   const float2* __restrict__ R, float2* __restrict__ M, int64_t ldM, int64_t strideS,
                   int64_t strideM, int batch) {
    extern __shared__ float2 lds[];
    using Fft = StaticFft<N, C, NT, R0, Rm...>;
    constexpr int NB = Fft::NB;
    int tile, item;
    tile_item(xcd_tile(blockIdx.x, gridDim.x), (F + C - 1) / C, batch, C, tile, item);
    S += (int64_t)item * strideS;
    M += (int64_t)item * strideM;
    const int j = threadIdx.x / C, s = threadIdx.x % C, f0 = tile * C;   // StaticFft's (j, s)
    const int f = min(f0 + s, F - 1);
    const bool f_ok = f0 + s < F;
    float2 v[R0], rr[R0], acc[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) acc[r] = make_float2(0.f, 0.f);
    // the gathers are unconditional (clamped rows, values masked at use) so
    // that a thread's loads are in flight together; the row index passes
    // through an empty asm so that the addresses are rebuilt per gather
    // rather than held in registers across the offset loop
    auto gather_s = [&](int k) {
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            int p = j + NB * r;
            asm volatile("" : "+v"(p));
            v[r] = S[(int64_t)(min(p, n_wires - 1) * n_imp + k) * ldS + f];
        }
    };
    auto gather_r = [&](int k) {
        const float2* Rk = R + (int64_t)k * N * F;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            int p = j + NB * r;
            asm volatile("" : "+v"(p));
            rr[r] = Rk[(int64_t)p * F + f];
        }
    };
    // the first gathers are in flight while the twiddle table is built
    gather_s(0);
    if (PREF) gather_r(0);
    Fft fx(lds, plan, threadIdx.x);
    for (int k = 0; k < n_imp; ++k) {
        float2 x[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const bool ok = f_ok && j + NB * r < n_wires;
            x[r] = ok ? v[r] : make_float2(0.f, 0.f);
        }
        if (k + 1 < n_imp) gather_s(k + 1);
        fx.run(x, false);
        if (!PREF) gather_r(k);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            acc[r].x += x[r].x * rr[r].x - x[r].y * rr[r].y;
            acc[r].y += x[r].x * rr[r].y + x[r].y * rr[r].x;
        }
        if (PREF && k + 1 < n_imp) gather_r(k + 1);
    }
    fx.run(acc, true);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int p = j + NB * r;
        if (p < n_wires && f_ok) M[(int64_t)p * ldM + f0 + s] = acc[r];
    }
}

// Wf = 512 with the plan 8 8 8 and T = 64 C takes k_wire_static.
static bool plan_is_888(const FftPlan& plan) {
    return plan.n == 512 && plan.npass == 3 && plan.radix[0] == 8 && plan.radix[1] == 8 && plan.radix[2] == 8;
}
static size_t static_lds_bytes(const FftPlan& plan, int C) {   // as StaticFft::lds_bytes
    return (size_t)(2 * (plan.n * C + plan.n * C / 32) + pm_entries(plan)) * sizeof(float2);
}

template <int C>
static hipError_t wire_launch_888(const float2* S, int64_t ldS, int n_wires, int n_imp, int F,
                                  const FftPlan& plan, const float2* R, float2* M, int64_t ldM, int batch,
                                  int64_t strideS, int64_t strideM, hipStream_t s) {
    const size_t lds = static_lds_bytes(plan, C);
    dim3 grid((unsigned)(((F + C - 1) / C) * batch)), block(64 * C);
    auto kern = k_wire_static<512, C, 64 * C, true, 8, 8>;
    set_lds(kern, lds);
    hipLaunchKernelGGL(kern, grid, block, lds, s, S, ldS, n_wires, n_imp, F, plan, R, M, ldM, strideS, strideM,
                       batch);
    return hipGetLastError();
}

// Wf = 864 with the plan 6 4 6 6 (radix order 5), 4 columns x 576 threads,
// takes k_wire_static without the response prefetch.
static bool plan_is_6466(const FftPlan& plan) {
    return plan.n == 864 && plan.npass == 4 && plan.radix[0] == 6 && plan.radix[1] == 4 && plan.radix[2] == 6 &&
           plan.radix[3] == 6;
}

static hipError_t wire_launch_6466(const float2* S, int64_t ldS, int n_wires, int n_imp, int F,
                                   const FftPlan& plan, const float2* R, float2* M, int64_t ldM, int batch,
                                   int64_t strideS, int64_t strideM, hipStream_t s) {
    constexpr int C = 4, NT = 576;
    const size_t lds = static_lds_bytes(plan, C);
    dim3 grid((unsigned)(((F + C - 1) / C) * batch)), block(NT);
    auto kern = k_wire_static<864, C, NT, false, 6, 4, 6>;
    set_lds(kern, lds);
    hipLaunchKernelGGL(kern, grid, block, lds, s, S, ldS, n_wires, n_imp, F, plan, R, M, ldM, strideS, strideM,
                       batch);
    return hipGetLastError();
}

template <int VPT, int C, int NT>
static hipError_t wire_launch(const float2* S, int64_t ldS, int n_wires, int n_imp, int F,
                              const FftPlan& plan, const float2* R, float2* M, int64_t ldM,
                              int batch, int64_t strideS, int64_t strideM, hipStream_t s) {
    const size_t lds = wire_lds_bytes(plan, C);
    dim3 grid((unsigned)(((F + C - 1) / C) * batch)), block(NT);
    // the first pass in registers when each thread holds one butterfly's inputs
    const bool reg = plan.radix[0] == VPT && NT * VPT == plan.n * C;
#define LAR_WF(RG, S6)                                                                                  \
    {                                                                                                   \
        set_lds(k_wire_fused<VPT, C, NT, RG, S6>, lds);                                                 \
        hipLaunchKernelGGL((k_wire_fused<VPT, C, NT, RG, S6>), grid, block, lds, s, S, ldS, n_wires, n_imp, \
                           F, plan, R, M, ldM, strideS, strideM, batch);                                \
    }
    if (plan_has6(plan)) LAR_WF(0, true)
    else if (reg) LAR_WF(1, false)
    else LAR_WF(0, false)
#undef LAR_WF
    return hipGetLastError();
}

// Default wire tiles: 16 columns x 1024 threads for Wf = 512 (k_wire_static,
// whole 128-byte row segments), 4 x 576 with radix order 5 for Wf = 864
// (k_wire_static, 6 4 6 6), 8 x 512 below 512, 4 x 512 otherwise (more
// resident workgroups per CU).
int default_wire_cols(int nw_fft) { return nw_fft == 512 ? 16 : (nw_fft < 512 ? 8 : 4); }
int default_wire_threads(int nw_fft) { return nw_fft == 512 ? 1024 : (nw_fft == 864 ? 576 : 512); }
int default_wire_order(int nw_fft) { return nw_fft == 864 ? 5 : 0; }

bool wire_sched_ok(int nw_fft, int cols, int threads, int order) {
    FftPlan plan;
    if (cols == 4 && threads == 576)   // k_wire_static with the 6 4 6 6 plan only
        return make_plan(nw_fft, &plan, order) && plan_is_6466(plan) && static_lds_bytes(plan, 4) <= kLdsBytes;
    const bool shape = (cols == 4 && (threads == 256 || threads == 512)) ||
                       (cols == 8 && (threads == 256 || threads == 512 || threads == 1024)) ||
                       (cols == 16 && (threads == 512 || threads == 1024));
    // the tile and its twiddle tables must fit the 160 KB of LDS of a CU
    if (!shape || !vpt_for(nw_fft * cols, threads) || !make_plan(nw_fft, &plan, order)) return false;
    if (plan_is_888(plan) && threads == 64 * cols)   // k_wire_static: two [Wf][C] buffers
        return static_lds_bytes(plan, cols) <= kLdsBytes;
    return wire_lds_bytes(plan, cols) <= kLdsBytes;
}

// Tiles of C time-frequency columns (neighbouring tiles run on one XCD and
// share its L2 lines) by T threads, so that a thread holds at most 8 values
// per tile array; defaults as default_wire_cols / default_wire_threads.
hipError_t launch_wire_fused(const float2* S, int64_t ldS, int n_wires, int n_imp, int nw_fft,
                             int F, const float2* R, float2* M, int64_t ldM, hipStream_t s,
                             int batch, int64_t strideS, int64_t strideM, int cols, int threads,
                             int order) {
    if (!cols) {
        cols = default_wire_cols(nw_fft);
        threads = default_wire_threads(nw_fft);
        order = default_wire_order(nw_fft);
    }
    if (!threads) threads = default_wire_threads(nw_fft);
    FftPlan plan;
    if (!wire_sched_ok(nw_fft, cols, threads, order) || !make_plan(nw_fft, &plan, order))
        return hipErrorInvalidValue;
    if (F <= 0 || batch <= 0) return hipSuccess;
    if (plan_is_6466(plan) && cols == 4 && threads == 576)
        return wire_launch_6466(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, batch, strideS, strideM, s);
    if (plan_is_888(plan) && threads == 64 * cols) {
        if (cols == 4) return wire_launch_888<4>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, batch, strideS, strideM, s);
        if (cols == 8) return wire_launch_888<8>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, batch, strideS, strideM, s);
        if (cols == 16) return wire_launch_888<16>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, batch, strideS, strideM, s);
    }
    const int vpt = vpt_for(nw_fft * cols, threads);
#define LAR_W(V, C, T)                                                                          \
    case (C) * 100000 + (T) * 16 + (V):                                                         \
        return wire_launch<V, C, T>(S, ldS, n_wires, n_imp, F, plan, R, M, ldM, batch, strideS, \
                                    strideM, s);
#define LAR_W4(C, T) LAR_W(1, C, T) LAR_W(2, C, T) LAR_W(4, C, T) LAR_W(8, C, T)
    switch (cols * 100000 + threads * 16 + vpt) {
        LAR_W4(4, 256)
        LAR_W4(4, 512)
        LAR_W4(8, 256)
        LAR_W4(8, 512)
        LAR_W4(8, 1024)
        LAR_W4(16, 512)
        LAR_W4(16, 1024)
        default: return hipErrorInvalidValue;
    }
#undef LAR_W4
#undef LAR_W
}

// ---------------------------------------------------------------- wire pass, adjoint
//
// For a tile of C time-frequency columns: Gh = FFT over wires of the
// waveform-gradient spectrum Gt (rows w < n_wires, zero padded).  For each
// impact offset k:
//  - response gradient (dR != null): Sk = FFT over wires of the grid
//    spectrum rows w*n_imp + k, dR[k] += resp_scale c_f Gh conj(Sk), with
//    c_f = 1 at f = 0 and f = Tf/2 and 2 elsewhere;
//  - grid gradient (want_grid): conj(R[k]) Gh, inverse FFT over wires,
//    written to the rows w*n_imp + k of O.  O may be S itself: each tile
//    reads its columns of a row of S before it writes them.
template <int VPT, int C, int NT>
__global__ __launch_bounds__(NT) void k_wire_adjoint(
    const float2* __restrict__ Gt, int64_t ldG, const float2* S, int64_t ldS, float2* O, int64_t ldO,
    int n_wires, int n_imp, int F, int nyq, FftPlan plan, const float2* __restrict__ R,
    float2* __restrict__ dR, int want_grid, float resp_scale, int accumulate) {
    extern __shared__ float2 lds[];
    const int Wf = plan.n, tid = threadIdx.x, T = NT;
    float2* A = lds;
    float2* tw = lds + Wf * C;
    fill_full_table(tw, Wf, tid, T);
    const TwFull twf{tw};
    const int f0 = xcd_tile(blockIdx.x, gridDim.x) * C;
    const int nel = Wf * C;
    float2 gh[VPT];
    // ---- Gh
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        const int e = tid + i * T;
        const int p = e / C, f = f0 + e % C;
        const bool ok = e < nel && p < n_wires && f < F;
        const float2 v = Gt[(int64_t)min(p, n_wires - 1) * ldG + min(f, F - 1)];
        gh[i] = ok ? v : make_float2(0.f, 0.f);
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        const int e = tid + i * T;
        if (e < nel) A[e] = gh[i];
    }
    lds_barrier();
    fft_lds<VPT, C>(A, plan, tid, T, twf, false);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        const int e = tid + i * T;
        if (e < nel) gh[i] = A[e];
    }
    for (int k = 0; k < n_imp; ++k) {
        if (dR) {
            float2 v[VPT];
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                const int p = e / C, f = f0 + e % C;
                const bool ok = e < nel && p < n_wires && f < F;
                const float2 x = S[(int64_t)(min(p, n_wires - 1) * n_imp + k) * ldS + min(f, F - 1)];
                v[i] = ok ? x : make_float2(0.f, 0.f);
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                if (e < nel) A[e] = v[i];
            }
            lds_barrier();
            fft_lds<VPT, C>(A, plan, tid, T, twf, false);
            float2* dRk = dR + (int64_t)k * Wf * F;
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                const int p = e / C, f = f0 + e % C;
                if (e < nel && f < F) {
                    const float cf = (f == 0 || f == nyq) ? resp_scale : 2.f * resp_scale;
                    const float2 sk = A[e];
                    const float2 g = cmulc(gh[i], sk);   // Gh conj(Sk)
                    float2* o = dRk + (int64_t)p * F + f;
                    float2 cur = accumulate ? *o : make_float2(0.f, 0.f);
                    cur.x += cf * g.x;
                    cur.y += cf * g.y;
                    *o = cur;
                }
            }
        }
        if (want_grid) {
            const float2* Rk = R + (int64_t)k * Wf * F;
            float2 r[VPT];
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                const int p = min(e / C, Wf - 1), f = min(f0 + e % C, F - 1);
                r[i] = Rk[(int64_t)p * F + f];
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                if (e < nel) A[e] = cmulc(gh[i], r[i]);   // conj(R) Gh
            }
            lds_barrier();
            fft_lds<VPT, C>(A, plan, tid, T, twf, true);
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                const int p = e / C, f = f0 + e % C;
                if (e < nel && p < n_wires && f < F) O[(int64_t)(p * n_imp + k) * ldO + f] = A[e];
            }
        }
    }
}

// k_wire_adjoint with a compile-time plan (StaticFft): thread (j, s) holds
// the wires / wire frequencies j + (N / R0) r of column s throughout, so
// Gh, each offset's grid-spectrum transform and their products never leave
// registers, and the next offset's rows are requested before this offset's
// transforms.
template <int N, int C, int NT, int R0, int... Rm>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_wire_adjoint_static(const float2* __restrict__ Gt, int64_t ldG, const float2* S, int64_t ldS, float2* O,
                           int64_t ldO, int n_wires, int n_imp, int F, int nyq, FftPlan plan,
                           const float2* __restrict__ R, float2* __restrict__ dR, int want_grid, float resp_scale,
                           int accumulate) {
    extern __shared__ float2 lds[];
    using Fft = StaticFft<N, C, NT, R0, Rm...>;
    constexpr int NB = Fft::NB;
    Fft fx(lds, plan, threadIdx.x);
    const int j = fx.j, s = fx.s, f0 = xcd_tile(blockIdx.x, gridDim.x) * C;
    const int f = min(f0 + s, F - 1);
    const bool f_ok = f0 + s < F;
    const float cf = (f0 + s == 0 || f0 + s == nyq) ? resp_scale : 2.f * resp_scale;
    float2 gh[R0], v[R0], rr[R0];
    // unconditional gathers (clamped rows, masked at use), as in k_wire_static
    auto gather = [&](float2 (&x)[R0], const float2* base, int64_t ld, int rstride, int off) {
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            int p = j + NB * r;
            asm volatile("" : "+v"(p));
            x[r] = base[(int64_t)(min(p, n_wires - 1) * rstride + off) * ld + f];
        }
    };
    auto masked = [&](float2 (&x)[R0], const float2 (&y)[R0]) {
#pragma unroll
        for (int r = 0; r < R0; ++r) x[r] = (f_ok && j + NB * r < n_wires) ? y[r] : make_float2(0.f, 0.f);
    };
    auto gather_r = [&](int k) {
        const float2* Rk = R + (int64_t)k * N * F;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            int p = j + NB * r;
            asm volatile("" : "+v"(p));
            rr[r] = Rk[(int64_t)p * F + f];
        }
    };
    gather(v, Gt, ldG, 1, 0);
    masked(gh, v);
    if (dR) gather(v, S, ldS, n_imp, 0);
    if (want_grid) gather_r(0);
    fx.run(gh, false);
    for (int k = 0; k < n_imp; ++k) {
        if (dR) {
            float2 x[R0];
            masked(x, v);
            if (k + 1 < n_imp) gather(v, S, ldS, n_imp, k + 1);
            fx.run(x, false);
            float2* dRk = dR + (int64_t)k * N * F;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                if (f_ok) {
                    float2* o = dRk + (int64_t)(j + NB * r) * F + f0 + s;
                    const float2 g = cmulc(gh[r], x[r]);   // Gh conj(Sk)
                    float2 cur = accumulate ? *o : make_float2(0.f, 0.f);
                    cur.x += cf * g.x;
                    cur.y += cf * g.y;
                    *o = cur;
                }
            }
        }
        if (want_grid) {
            float2 y[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) y[r] = cmulc(gh[r], rr[r]);   // conj(R) Gh
            if (k + 1 < n_imp) gather_r(k + 1);
            fx.run(y, true);
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int p = j + NB * r;
                if (p < n_wires && f_ok) O[(int64_t)(p * n_imp + k) * ldO + f0 + s] = y[r];
            }
        }
    }
}

// The batched adjoint wire pass with a compile-time plan (StaticFft): one
// workgroup per (column tile, KG consecutive impact offsets), the items of
// the batch as its inner loop.  Each item's Gh (the wire transform of its
// waveform-gradient tile) is formed once per workgroup and serves the KG
// offsets; their response gradients are summed over the items in registers
// and written once, so no partial sums are needed; item b's grid-gradient
// spectrum is written over its S rows (each row of offset k is read, for
// the response gradient, before it is written, by the same thread).  PF:
// the next item's Gt rows are requested before this item's transforms.
template <int N, int C, int NT, int KG, bool PF, int R0, int... Rm>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_wire_adjoint_offsets_static(const float2* __restrict__ Gt, int64_t ldG, int64_t strideG, float2* S,
                                   int64_t ldS, int64_t strideS, int batch, int n_wires, int n_imp, int F,
                                   int nyq, FftPlan plan, const float2* __restrict__ R, float2* __restrict__ dR,
                                   float resp_scale, int accumulate) {
    extern __shared__ float2 lds[];
    using Fft = StaticFft<N, C, NT, R0, Rm...>;
    constexpr int NB = Fft::NB;
    Fft fx(lds, plan, threadIdx.x);
    int tile, kg;
    tile_item(xcd_tile(blockIdx.x, gridDim.x), (F + C - 1) / C, (n_imp + KG - 1) / KG, C, tile, kg);
    const int k0 = kg * KG, nk = min(KG, n_imp - k0);
    const int j = fx.j, s = fx.s, f0 = tile * C;
    const int f = min(f0 + s, F - 1);
    const bool f_ok = f0 + s < F;
    const float cf = (f0 + s == 0 || f0 + s == nyq) ? resp_scale : 2.f * resp_scale;
    // unconditional gathers (clamped rows, masked at use), as in k_wire_static
    auto gather = [&](float2 (&x)[R0], const float2* base, int64_t ld, int rstride, int off) {
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            int p = j + NB * r;
            asm volatile("" : "+v"(p));
            x[r] = base[(int64_t)(min(p, n_wires - 1) * rstride + off) * ld + f];
        }
    };
    auto masked = [&](float2 (&x)[R0]) {
#pragma unroll
        for (int r = 0; r < R0; ++r) x[r] = (f_ok && j + NB * r < n_wires) ? x[r] : make_float2(0.f, 0.f);
    };
    float2 dacc[KG][R0], g[R0];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int r = 0; r < R0; ++r) dacc[kk][r] = make_float2(0.f, 0.f);
    if (PF && batch > 0) gather(g, Gt, ldG, 1, 0);
    for (int b = 0; b < batch; ++b) {
        float2* Sb = S + (int64_t)b * strideS;
        float2 gh[R0];
        if (!PF) gather(g, Gt + (int64_t)b * strideG, ldG, 1, 0);
#pragma unroll
        for (int r = 0; r < R0; ++r) gh[r] = g[r];
        masked(gh);
        if (PF && b + 1 < batch) gather(g, Gt + (int64_t)(b + 1) * strideG, ldG, 1, 0);
        fx.run(gh, false);
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            if (kk >= nk) break;   // workgroup-uniform
            const int k = k0 + kk;
            float2 x[R0];
            if (dR) {
                gather(x, Sb, ldS, n_imp, k);
                masked(x);
                fx.run(x, false);
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const float2 q = cmulc(gh[r], x[r]);   // Gh conj(Sk)
                    dacc[kk][r].x += q.x;
                    dacc[kk][r].y += q.y;
                }
            }
            const float2* Rk = R + (int64_t)k * N * F;
#pragma unroll
            for (int r = 0; r < R0; ++r) x[r] = cmulc(gh[r], Rk[(int64_t)(j + NB * r) * F + f]);   // conj(R) Gh
            fx.run(x, true);
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int p = j + NB * r;
                if (p < n_wires && f_ok) Sb[(int64_t)(p * n_imp + k) * ldS + f0 + s] = x[r];
            }
        }
    }
    if (dR && f_ok) {
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            if (kk >= nk) break;
            float2* dRk = dR + (int64_t)(k0 + kk) * N * F;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                float2* o = dRk + (int64_t)(j + NB * r) * F + f0 + s;
                float2 cur = accumulate ? *o : make_float2(0.f, 0.f);
                cur.x += cf * dacc[kk][r].x;
                cur.y += cf * dacc[kk][r].y;
                *o = cur;
            }
        }
    }
}

template <int VPT, int C, int NT>
static hipError_t wire_adj_launch(const float2* Gt, int64_t ldG, const float2* S, int64_t ldS,
                                  float2* O, int64_t ldO, int n_wires, int n_imp, int F, int nyq,
                                  const FftPlan& plan, const float2* R, float2* dR, bool want_grid,
                                  float scale, bool accumulate, hipStream_t s) {
    const size_t lds = ((size_t)plan.n * C + plan.n) * sizeof(float2);
    set_lds(k_wire_adjoint<VPT, C, NT>, lds);
    dim3 grid((F + C - 1) / C), block(NT);
    hipLaunchKernelGGL((k_wire_adjoint<VPT, C, NT>), grid, block, lds, s, Gt, ldG, S, ldS, O, ldO,
                       n_wires, n_imp, F, nyq, plan, R, dR, want_grid ? 1 : 0, scale,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_wire_adjoint(const float2* Gt, int64_t ldG, const float2* S, int64_t ldS, float2* O,
                               int64_t ldO, int n_wires, int n_imp, int nw_fft, int nt_fft,
                               const float2* R, float2* dR, bool want_grid, float resp_scale,
                               hipStream_t s, bool accumulate) {
    FftPlan plan;
    if (!make_plan(nw_fft, &plan)) return hipErrorInvalidValue;
    const int F = nt_fft / 2 + 1, nyq = nt_fft / 2;
    if (plan_is_888(plan)) {   // 16 columns x 1024 threads, as the forward pass's default
        constexpr int C = 16;
        auto kern = k_wire_adjoint_static<512, C, 64 * C, 8, 8>;
        const size_t lds = static_lds_bytes(plan, C);
        set_lds(kern, lds);
        hipLaunchKernelGGL(kern, dim3((F + C - 1) / C), dim3(64 * C), lds, s, Gt, ldG, S, ldS, O, ldO, n_wires,
                           n_imp, F, nyq, plan, R, dR, want_grid ? 1 : 0, resp_scale, accumulate ? 1 : 0);
        return hipGetLastError();
    }
#define LAR_WADJ(V)                                                                                   \
    return wire_adj_launch<V, 8, 512>(Gt, ldG, S, ldS, O, ldO, n_wires, n_imp, F, nyq, plan, R, dR,   \
                                      want_grid, resp_scale, accumulate, s);
    if (nw_fft <= 128) LAR_WADJ(2)
    if (nw_fft <= 256) LAR_WADJ(4)
    if (nw_fft <= 512) LAR_WADJ(8)
    if (nw_fft <= 1024)
        return wire_adj_launch<8, 8, 1024>(Gt, ldG, S, ldS, O, ldO, n_wires, n_imp, F, nyq, plan, R,
                                           dR, want_grid, resp_scale, accumulate, s);
#undef LAR_WADJ
    return hipErrorInvalidValue;
}

// The adjoint wire pass over a batch of items sharing one response (the
// batch plan's backward): per tile and impact offset k, the items are the
// inner loop, so the response-spectrum gradient of the tile is summed over
// the items in registers and written once per k, and R[k] is read once per
// tile.  The items are split into `groups` consecutive ranges, one block per
// (tile, group) (groups of one tile run together on one XCD); with one group
// the sum goes to dR (= or += with accumulate), else group g writes its sum
// to part + g * part_stride, for k_sum_parts.  Each item's Gh is the wire
// FFT of its Gt tile, recomputed per k (its rows are re-read from L2) rather
// than held for every item.  The grid-gradient spectrum of item b is
// written over its S rows (each tile reads them first).  Item b's arrays are
// at Gt + b*strideG and S + b*strideS.
template <int VPT, int C, int NT>
__global__ __launch_bounds__(NT) void k_wire_adjoint_items(
    const float2* __restrict__ Gt, int64_t ldG, int64_t strideG, float2* S, int64_t ldS, int64_t strideS,
    int batch, int groups, int n_wires, int n_imp, int F, int nyq, FftPlan plan, const float2* __restrict__ R,
    float2* __restrict__ dR, float2* __restrict__ part, int64_t part_stride, float resp_scale, int accumulate) {
    extern __shared__ float2 lds[];
    const int Wf = plan.n, tid = threadIdx.x, T = NT;
    float2* A = lds;
    float2* tw = lds + Wf * C;
    fill_full_table(tw, Wf, tid, T);
    const TwFull twf{tw};
    int tile, grp;
    tile_item(xcd_tile(blockIdx.x, gridDim.x), (F + C - 1) / C, groups, C, tile, grp);
    const int per = (batch + groups - 1) / groups;
    const int b0 = grp * per, b1 = min(batch, b0 + per);
    if (groups > 1 && dR) {
        dR = part + (int64_t)grp * part_stride;
        accumulate = 0;
    }
    const int f0 = tile * C;
    const int nel = Wf * C;
    // load a [wire][column] tile of rows p * rstride + off into A (zero outside)
    auto load_tile = [&](const float2* base, int64_t ld, int rstride, int off, int rows) {
        float2 v[VPT];
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + i * T;
            const int p = e / C, f = f0 + e % C;
            const bool ok = e < nel && p < rows && f < F;
            const float2 x = base[(int64_t)(min(p, rows - 1) * rstride + off) * ld + min(f, F - 1)];
            v[i] = ok ? x : make_float2(0.f, 0.f);
        }
        lds_barrier();
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + i * T;
            if (e < nel) A[e] = v[i];
        }
        lds_barrier();
    };
    for (int k = 0; k < n_imp; ++k) {
        float2 dacc[VPT], r[VPT];
        const float2* Rk = R + (int64_t)k * Wf * F;
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            dacc[i] = make_float2(0.f, 0.f);
            const int e = tid + i * T;
            const int p = min(e / C, Wf - 1), f = min(f0 + e % C, F - 1);
            r[i] = Rk[(int64_t)p * F + f];
        }
        for (int b = b0; b < b1; ++b) {
            const float2* Gb = Gt + (int64_t)b * strideG;
            float2* Sb = S + (int64_t)b * strideS;
            float2 gh[VPT];
            load_tile(Gb, ldG, 1, 0, n_wires);
            fft_lds<VPT, C>(A, plan, tid, T, twf, false);
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                if (e < nel) gh[i] = A[e];
            }
            if (dR) {
                load_tile(Sb, ldS, n_imp, k, n_wires);
                fft_lds<VPT, C>(A, plan, tid, T, twf, false);
#pragma unroll
                for (int i = 0; i < VPT; ++i) {
                    const int e = tid + i * T;
                    if (e < nel) {
                        const float2 g = cmulc(gh[i], A[e]);   // Gh conj(Sk)
                        dacc[i].x += g.x;
                        dacc[i].y += g.y;
                    }
                }
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                if (e < nel) A[e] = cmulc(gh[i], r[i]);   // conj(R) Gh
            }
            lds_barrier();
            fft_lds<VPT, C>(A, plan, tid, T, twf, true);
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                const int p = e / C, f = f0 + e % C;
                if (e < nel && p < n_wires && f < F) Sb[(int64_t)(p * n_imp + k) * ldS + f] = A[e];
            }
        }
        if (dR) {
            float2* dRk = dR + (int64_t)k * Wf * F;
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int e = tid + i * T;
                const int p = e / C, f = f0 + e % C;
                if (e < nel && f < F) {
                    const float cf = (f == 0 || f == nyq) ? resp_scale : 2.f * resp_scale;
                    float2* o = dRk + (int64_t)p * F + f;
                    float2 cur = accumulate ? *o : make_float2(0.f, 0.f);
                    cur.x += cf * dacc[i].x;
                    cur.y += cf * dacc[i].y;
                    *o = cur;
                }
            }
        }
    }
}

// dR[i] = (accumulate ? dR[i] : 0) + sum_g part[g * stride + i], i < n, in group order.
__global__ __launch_bounds__(256) void k_sum_parts(float2* __restrict__ dR, const float2* __restrict__ part,
                                                   int64_t stride, int groups, int64_t n, int accumulate) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        float2 a = accumulate ? dR[i] : make_float2(0.f, 0.f);
        for (int g = 0; g < groups; ++g) {
            const float2 v = part[(int64_t)g * stride + i];
            a.x += v.x;
            a.y += v.y;
        }
        dR[i] = a;
    }
}

int wire_adjoint_groups(int batch, size_t scratch_bytes, int n_imp, int nw_fft, int nt_fft) {
    const size_t one = (size_t)n_imp * nw_fft * (nt_fft / 2 + 1) * sizeof(float2);
    int g = batch < kAdjointGroups ? batch : kAdjointGroups;
    while (g > 1 && (size_t)g * one > scratch_bytes) --g;
    return g < 1 ? 1 : g;
}

hipError_t launch_wire_adjoint_items(const float2* Gt, int64_t ldG, int64_t strideG, float2* S, int64_t ldS,
                                     int64_t strideS, int batch, int n_wires, int n_imp, int nw_fft,
                                     int nt_fft, const float2* R, float2* dR, float resp_scale,
                                     hipStream_t s, bool accumulate, void* scratch, size_t scratch_bytes) {
    FftPlan plan;
    if (!make_plan(nw_fft, &plan)) return hipErrorInvalidValue;
    if (batch <= 0) return hipSuccess;
    const int F = nt_fft / 2 + 1, nyq = nt_fft / 2;
    const int groups = dR ? wire_adjoint_groups(batch, scratch ? scratch_bytes : 0, n_imp, nw_fft, nt_fft)
                          : (batch < kAdjointGroups ? batch : kAdjointGroups);
    const int64_t pstride = (int64_t)n_imp * nw_fft * F;
    float2* part = reinterpret_cast<float2*>(scratch);
    constexpr int C = 8;
    if (plan_is_888(plan)) {
        // one impact offset per workgroup, every item in each: no partials.
        // (With two offsets per workgroup, sharing each Gh, the two response
        // gradient sums spill registers: slower, measured.)
        constexpr int KG = 1;
        auto kern = k_wire_adjoint_offsets_static<512, C, 64 * C, KG, true, 8, 8>;
        const size_t lds8 = static_lds_bytes(plan, C);
        set_lds(kern, lds8);
        const dim3 grid8((unsigned)(((F + C - 1) / C) * ((n_imp + KG - 1) / KG)));
        hipLaunchKernelGGL(kern, grid8, dim3(64 * C), lds8, s, Gt, ldG, strideG, S, ldS, strideS, batch, n_wires,
                           n_imp, F, nyq, plan, R, dR, resp_scale, accumulate ? 1 : 0);
        return hipGetLastError();
    }
    dim3 grid((unsigned)(((F + C - 1) / C) * groups));
    hipError_t e = hipErrorInvalidValue;
    const size_t lds = ((size_t)plan.n * C + plan.n) * sizeof(float2);
#define LAR_WADJI(V, NT)                                                                                \
    {                                                                                                   \
        set_lds(k_wire_adjoint_items<V, C, NT>, lds);                                                   \
        hipLaunchKernelGGL((k_wire_adjoint_items<V, C, NT>), grid, dim3(NT), lds, s, Gt, ldG, strideG, S, \
                           ldS, strideS, batch, groups, n_wires, n_imp, F, nyq, plan, R, dR, part,      \
                           pstride, resp_scale, accumulate ? 1 : 0);                                    \
        e = hipGetLastError();                                                                          \
    }
    if (nw_fft <= 128) LAR_WADJI(2, 512)
    else if (nw_fft <= 256) LAR_WADJI(4, 512)
    else if (nw_fft <= 512) LAR_WADJI(8, 512)
    else if (nw_fft <= 1024) LAR_WADJI(8, 1024)
#undef LAR_WADJI
    if (e != hipSuccess || !dR || groups == 1) return e;
    const int64_t b = (pstride + 255) / 256, cap = 8 * (int64_t)device_cus();
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)(b < cap ? b : cap)), dim3(256), 0, s, dR, part, pstride, groups,
                       pstride, accumulate ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------- response spectrum
//
// rows: time spectra [n_imp][nrw][ld_rows] of the response rows (dw = row -
// half_w); resp[k][p][f] = sum over rows with dw mod Wf = p, then a forward
// FFT over p.
template <int VPT, int C>
__global__ __launch_bounds__(256) void k_wire_spectrum(
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
    dim3 grid((F + C - 1) / C, n_imp), block(256);
    if (nw_fft * C <= 8 * 256) {
        set_lds(k_wire_spectrum<8, C>, lds);
        hipLaunchKernelGGL((k_wire_spectrum<8, C>), grid, block, lds, s, rows, ld_rows, nrw,
                           half_w, F, plan, resp);
    } else if (nw_fft * C <= 32 * 256) {
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
