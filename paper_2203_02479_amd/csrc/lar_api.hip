// lar_api.hip -- host implementation of the C ABI declared in include/lar.h.
// Argument checks, workspace layout, kernel sequencing.  Everything is
// asynchronous on the caller's stream; nothing here allocates or syncs.
#include <limits.h>
#include <math.h>

#include <mutex>
#include <vector>

#include "lar_internal.hpp"

using namespace lar;

namespace lar {
// probe_kernels.hip: n_seg scattered 64-float atomic segments into buf.
hipError_t launch_atomic_probe(float* buf, int64_t n_floats, int64_t n_seg, hipStream_t s);
// probe_kernels.hip: Philox blocks and uniforms, one sum per thread.
hipError_t launch_philox_probe(double* out, int64_t n_threads, int64_t n_blocks, hipStream_t s);
// probe_kernels.hip: the time R2C's row access pattern without the transform.
hipError_t launch_row_copy_probe(const float* in, int64_t ld_in, int n_in, int nrows, float2* out, int64_t ld_out,
                                 int n_out, int per_cu, hipStream_t s);
}

static thread_local int g_last_hip = 0;
static thread_local hipEvent_t g_stage_ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

static hipError_t stage_mark(int i, hipStream_t s) {
    return g_stage_ev[i] ? hipEventRecord(g_stage_ev[i], s) : hipSuccess;
}

static int hip_status(hipError_t e) {
    if (e == hipSuccess) return LAR_OK;
    g_last_hip = (int)e;
    return LAR_EHIP;
}

#define LAR_TRY(expr)                          \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return hip_status(_e); \
    } while (0)

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Row pitch (complex elements) of the internal time-spectrum buffers: the
// half spectrum padded to a multiple of 16 so rows start on 128-byte lines.
static int64_t spec_ld(const lar_plane* p) { return ((int64_t)(p->nt_fft / 2 + 1) + 15) / 16 * 16; }

static Sched sched_of(const lar_plane* p) {
    return sched_for(p->n_wires, p->n_imp, p->n_ticks, p->nt_fft, p->nw_fft);
}

static bool smooth(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

static int check_plane(const lar_plane* p) {
    if (!p) return LAR_EINVAL;
    if (p->n_wires < 1 || p->n_imp < 1 || p->n_ticks < 1) return LAR_EINVAL;
    if (!(p->tick > 0.f) || !(p->pitch > 0.f) || !isfinite(p->x0) || !isfinite(p->t0))
        return LAR_EINVAL;
    if ((int64_t)p->n_wires * p->n_imp > INT_MAX / 2) return LAR_ESIZE;
    return LAR_OK;
}

static int check_fft(const lar_plane* p) {
    int st = check_plane(p);
    if (st) return st;
    if (p->nt_fft % 2 || !smooth(p->nt_fft / 2) || p->nt_fft < p->n_ticks || p->nt_fft > 16384)
        return LAR_ESIZE;
    if (!smooth(p->nw_fft) || p->nw_fft < p->n_wires || p->nw_fft > 1024) return LAR_ESIZE;
    return LAR_OK;
}

static int check_depos(const lar_depos* d) {
    if (!d || d->n < 0) return LAR_EINVAL;
    if (d->n > 0 && (!d->q || !d->t || !d->x || !d->sigma_t || !d->sigma_x)) return LAR_EINVAL;
    if (d->n > (int64_t)UINT32_MAX) return LAR_ESIZE;   // depo index is one counter word
    return LAR_OK;
}

static int check_fluct(const lar_fluct* f, const lar_plane* p) {
    if (!f) return LAR_OK;
    if (f->mode < 0 || f->mode > 3) return LAR_EINVAL;
    if (f->plane >= 256u) return LAR_EINVAL;              // plane * 2^24 must fit one word
    // a drawn bin's counter word is m * n_ticks + j
    if (f->mode != 0 && (int64_t)p->n_wires * p->n_imp * p->n_ticks > (int64_t)UINT32_MAX)
        return LAR_ESIZE;
    return LAR_OK;
}

extern "C" {

const char* lar_status_str(int s) {
    switch (s) {
        case LAR_OK: return "ok";
        case LAR_EINVAL: return "invalid argument";
        case LAR_ESIZE: return "unsupported size";
        case LAR_EWORKSPACE: return "workspace missing or too small";
        case LAR_EHIP: return "HIP launch failed";
        default: return "unknown status";
    }
}

int lar_last_hip_error(void) { return g_last_hip; }

int lar_atomic_probe(float* buf, int64_t n_floats, int64_t n_segments, void* stream) {
    if (!buf || n_floats < 64 || n_segments < 0 || reinterpret_cast<uintptr_t>(buf) % 256) return LAR_EINVAL;
    LAR_TRY(launch_atomic_probe(buf, n_floats, n_segments, (hipStream_t)stream));
    return LAR_OK;
}

int lar_philox_probe(double* out, int64_t n_threads, int64_t n_blocks, void* stream) {
    if (!out || n_threads < 256 || n_threads % 256 || n_threads / 256 > INT_MAX || n_blocks < 0 ||
        reinterpret_cast<uintptr_t>(out) % 8)
        return LAR_EINVAL;
    LAR_TRY(launch_philox_probe(out, n_threads, n_blocks, (hipStream_t)stream));
    return LAR_OK;
}

int lar_row_copy_probe(const float* in, int64_t ld_in, int32_t n_in, int32_t n_rows, void* out, int64_t ld_out,
                       int32_t n_out, int32_t blocks_per_cu, void* stream) {
    if (n_rows < 0 || blocks_per_cu < 1 || blocks_per_cu > 16) return LAR_EINVAL;
    if (n_rows == 0) return LAR_OK;
    if (!in || !out || n_in < 2 || (n_in & 1) || n_in > 6144 || n_out < 1 || n_out > 3073 || ld_in < n_in ||
        ld_out < n_out || (ld_in & 1) || reinterpret_cast<uintptr_t>(in) % 8 || reinterpret_cast<uintptr_t>(out) % 8)
        return LAR_EINVAL;
    LAR_TRY(launch_row_copy_probe(in, ld_in, n_in, n_rows, static_cast<float2*>(out), ld_out, n_out, blocks_per_cu,
                                  (hipStream_t)stream));
    return LAR_OK;
}

int lar_set_stage_events(void* const* events, int32_t n_events) {
    if (!events) {
        for (int i = 0; i < 6; ++i) g_stage_ev[i] = nullptr;
        return LAR_OK;
    }
    if (n_events < 6) return LAR_EINVAL;
    for (int i = 0; i < 6; ++i)
        if (!events[i]) return LAR_EINVAL;
    for (int i = 0; i < 6; ++i) g_stage_ev[i] = (hipEvent_t)events[i];
    return LAR_OK;
}

static size_t raster_bytes_min(int64_t n, const lar_fluct* f) {
    if (!f || f->mode == 0 || n <= 0) return 0;
    return raster_ws_fixed(n);
}

// recommended: room for 48 deferred bins per depo (rejection-regime bins
// that the first sampler stage leaves; about 22 per depo on track depos of
// 2300 electrons) plus a margin
static size_t raster_bytes(int64_t n, const lar_fluct* f) {
    size_t fixed = raster_bytes_min(n, f);
    if (!fixed) return 0;
    if (f->mode == 3) return fixed;   // the normal approximation queues nothing
    return fixed + ((size_t)n * 48 + 4096) * kDeferredBytes;
}

int lar_raster_workspace(const lar_plane* plane, int64_t n_depos, const lar_fluct* fluct,
                         size_t* bytes) {
    int st;
    if ((st = check_plane(plane))) return st;
    if ((st = check_fluct(fluct, plane))) return st;
    if (n_depos < 0 || !bytes) return LAR_EINVAL;
    *bytes = raster_bytes(n_depos, fluct);
    return LAR_OK;
}

static int raster_impl(const lar_plane* plane, const lar_depos* depos, float nsigma,
                       const lar_fluct* fluct, float* grid, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
    RasterArgs a;
    a.n_ticks = plane->n_ticks;
    a.n_rows = plane->n_wires * plane->n_imp;
    a.ld = plane->n_ticks;
    a.org_t = (double)plane->t0;
    a.wd_t = (double)plane->tick;
    a.org_x = (double)plane->x0 - (double)plane->pitch / 2.0;
    a.wd_x = (double)plane->pitch / (double)plane->n_imp;
    a.nsig = (double)nsigma;
    a.mode = fluct ? fluct->mode : 0;
    a.event = fluct ? fluct->event : 0u;
    a.plane = fluct ? fluct->plane : 0u;
    a.seed = fluct ? fluct->seed : 0ull;
    LAR_TRY(launch_raster(a, depos->q, depos->t, depos->x, depos->sigma_t, depos->sigma_x,
                          depos->n, grid, ws, ws_bytes, stream, g_stage_ev[1], sched_of(plane).raster_tile));
    LAR_TRY(stage_mark(2, stream));
    return LAR_OK;
}

int lar_depos_nonfinite(const lar_depos* depos, int64_t* count, void* stream) {
    int st;
    if ((st = check_depos(depos))) return st;
    if (!count || reinterpret_cast<uintptr_t>(count) % 8) return LAR_EINVAL;   // a 64-bit atomic target
    LAR_TRY(launch_count_nonfinite(depos->q, depos->t, depos->x, depos->sigma_t, depos->sigma_x, depos->n, count,
                                   (hipStream_t)stream));
    return LAR_OK;
}

int lar_raster(const lar_plane* plane, const lar_depos* depos, float nsigma, const lar_fluct* fluct,
               float* grid, void* ws, size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_plane(plane))) return st;
    if ((st = check_depos(depos))) return st;
    if ((st = check_fluct(fluct, plane))) return st;
    if (!(nsigma > 0.f) || !isfinite(nsigma)) return LAR_EINVAL;
    if (depos->n == 0) return LAR_OK;
    if (!grid) return LAR_EINVAL;
    const size_t need = raster_bytes_min(depos->n, fluct);
    if (need && (!ws || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % 256)) return LAR_EWORKSPACE;
    return raster_impl(plane, depos, nsigma, fluct, grid, ws, ws_bytes, (hipStream_t)stream);
}

// fftconv workspace: [spectrum of grid rows: R_rows x ld][wire-pass output: N_w x ld]
static size_t fftconv_bytes(const lar_plane* p) {
    size_t ld = (size_t)spec_ld(p);
    size_t a = align_up((size_t)p->n_wires * p->n_imp * ld * sizeof(float2), 256);
    size_t b = align_up((size_t)p->n_wires * ld * sizeof(float2), 256);
    return a + b;
}

int lar_fftconv_workspace(const lar_plane* plane, size_t* bytes) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (!bytes) return LAR_EINVAL;
    *bytes = fftconv_bytes(plane);
    return LAR_OK;
}

static int fftconv_impl(const lar_plane* p, const float* grid, const float* resp, float* wave,
                        void* ws, hipStream_t s) {
    const int64_t ld = spec_ld(p);
    const int rows = p->n_wires * p->n_imp;
    const int F = p->nt_fft / 2 + 1;
    float2* Sh = reinterpret_cast<float2*>(ws);
    float2* Mh = reinterpret_cast<float2*>(
        reinterpret_cast<char*>(ws) + align_up((size_t)rows * ld * sizeof(float2), 256));
    const Sched sc = sched_of(p);
    LAR_TRY(launch_r2c_rows(grid, p->n_ticks, p->n_ticks, rows, p->nt_fft, Sh, ld, s, sc.row_threads,
                            sc.row_order));
    LAR_TRY(stage_mark(3, s));
    LAR_TRY(launch_wire_fused(Sh, ld, p->n_wires, p->n_imp, p->nw_fft, F,
                              reinterpret_cast<const float2*>(resp), Mh, ld, s, 1, 0, 0,
                              sc.wire_cols, sc.wire_threads, sc.wire_order));
    LAR_TRY(stage_mark(4, s));
    const float scale = (float)(1.0 / ((double)p->nw_fft * (double)p->nt_fft));
    LAR_TRY(launch_c2r_rows(Mh, ld, p->n_wires, p->nt_fft, wave, p->n_ticks, p->n_ticks, scale, s,
                            nullptr, false, sc.row_threads, sc.row_order));
    LAR_TRY(stage_mark(5, s));
    return LAR_OK;
}

int lar_fftconv(const lar_plane* plane, const float* grid, const float* resp, float* wave,
                void* ws, size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (!grid || !resp || !wave) return LAR_EINVAL;
    if (!ws || ws_bytes < fftconv_bytes(plane)) return LAR_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return LAR_EWORKSPACE;
    return fftconv_impl(plane, grid, resp, wave, ws, (hipStream_t)stream);
}

// ---- the convolution without a caller workspace, for callers that cannot
// allocate: its time and wire-pass spectra live in one file-scope device
// array.  In host code `scratch` names a host-side stand-in, so its device
// address is looked up once per device (with that device current) and only
// that address is ever handed to kernels.
static constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_on_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return LAR_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (!ptr) return LAR_EINVAL;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LAR_OK;
}

size_t lar_fftconv_noalloc_max_bytes(void) { return kScratchBytes; }

int lar_fftconv_noalloc(const lar_plane* plane, const float* grid, const float* resp, float* wave,
                        void* stream) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (!grid || !resp || !wave) return LAR_EINVAL;
    if (fftconv_bytes(plane) > kScratchBytes) return LAR_ESIZE;
    void* ws = nullptr;
    if ((st = scratch_on_current_device(&ws))) return st;
    return fftconv_impl(plane, grid, resp, wave, ws, (hipStream_t)stream);
}

// sim_plane workspace: [grid: R_rows x n_ticks floats][fftconv workspace]
static size_t grid_bytes(const lar_plane* p) {
    return align_up((size_t)p->n_wires * p->n_imp * p->n_ticks * sizeof(float), 256);
}

// sim_plane workspace: [grid: R_rows x n_ticks floats][fftconv workspace][raster workspace]
int lar_sim_plane_workspace(const lar_plane* plane, int64_t n_depos, const lar_fluct* fluct,
                            size_t* bytes) {
    int st;
    if ((st = check_fft(plane))) return st;
    if ((st = check_fluct(fluct, plane))) return st;
    if (n_depos < 0 || !bytes) return LAR_EINVAL;
    *bytes = grid_bytes(plane) + fftconv_bytes(plane) + raster_bytes(n_depos, fluct);
    return LAR_OK;
}

// lar_sim_plane after its argument checks
static int sim_plane_impl(const lar_plane* plane, const lar_depos* depos, float nsigma, const lar_fluct* fluct,
                          const float* resp, float* wave, void* ws, size_t ws_bytes, hipStream_t s) {
    int st;
    const size_t head = grid_bytes(plane) + fftconv_bytes(plane);
    char* w = reinterpret_cast<char*>(ws);
    float* grid = reinterpret_cast<float*>(w);
    LAR_TRY(launch_fill(grid, (int64_t)plane->n_wires * plane->n_imp * plane->n_ticks, s));
    LAR_TRY(stage_mark(0, s));
    if (depos->n > 0) {
        if ((st = raster_impl(plane, depos, nsigma, fluct, grid, w + head, ws_bytes - head, s)))
            return st;
    } else {
        LAR_TRY(stage_mark(1, s));
        LAR_TRY(stage_mark(2, s));
    }
    return fftconv_impl(plane, grid, resp, wave, w + grid_bytes(plane), s);
}

int lar_sim_plane(const lar_plane* plane, const lar_depos* depos, float nsigma,
                  const lar_fluct* fluct, const float* resp, float* wave, void* ws,
                  size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_fft(plane))) return st;
    if ((st = check_depos(depos))) return st;
    if ((st = check_fluct(fluct, plane))) return st;
    if (!(nsigma > 0.f) || !isfinite(nsigma)) return LAR_EINVAL;
    if (!resp || !wave) return LAR_EINVAL;
    const size_t need = grid_bytes(plane) + fftconv_bytes(plane) + raster_bytes_min(depos->n, fluct);
    if (!ws || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % 256) return LAR_EWORKSPACE;
    return sim_plane_impl(plane, depos, nsigma, fluct, resp, wave, ws, ws_bytes, (hipStream_t)stream);
}

// ---- independent plane simulations on several streams (the single-GPU
// form of the paper's several processes per GPU, Sec. 3.3)

// Events of this host thread's calls, created on first use and kept: a
// stream wait takes the event's record made before the wait, so recording
// the same event again in a later call leaves earlier waits unchanged.
static thread_local std::vector<hipEvent_t> g_stream_ev;

static int stream_events(int n, hipEvent_t** out) {
    while ((int)g_stream_ev.size() < n) {
        hipEvent_t e = nullptr;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return hip_status(r);
        g_stream_ev.push_back(e);
    }
    *out = g_stream_ev.data();
    return LAR_OK;
}

// workspace slice of one stream: the largest lar_sim_plane workspace of the items
static size_t streams_slice(const lar_plane* planes, int32_t n_types, const lar_batch_item* items, int32_t n_items,
                            const lar_fluct* fluct) {
    size_t m = 0;
    for (int i = 0; i < n_items; ++i) {
        const lar_plane* p = &planes[items[i].plane_type];
        const size_t b = grid_bytes(p) + fftconv_bytes(p) + raster_bytes(items[i].n_depos, fluct);
        m = b > m ? b : m;
    }
    (void)n_types;
    return align_up(m, 256);
}

static int streams_check(const lar_plane* planes, int32_t n_types, const lar_batch_item* items, int32_t n_items,
                         const lar_fluct* fluct, int32_t n_streams) {
    int st;
    if (!planes || n_types < 1 || !items || n_items < 0 || n_streams < 1 || n_streams > 64) return LAR_EINVAL;
    for (int t = 0; t < n_types; ++t) {
        if ((st = check_fft(&planes[t]))) return st;
        if ((st = check_fluct(fluct, &planes[t]))) return st;
    }
    for (int i = 0; i < n_items; ++i) {
        const lar_batch_item& it = items[i];
        if (it.plane_type < 0 || it.plane_type >= n_types || it.n_depos < 0 || it.depo_offset < 0 ||
            it.wave_offset < 0 || it.plane >= 256u)
            return LAR_EINVAL;
        if (it.n_depos > (int64_t)UINT32_MAX) return LAR_ESIZE;
    }
    return LAR_OK;
}

int lar_sim_streams_workspace(const lar_plane* planes, int32_t n_types, const lar_batch_item* items,
                              int32_t n_items, const lar_fluct* fluct, int32_t n_streams, size_t* bytes) {
    int st;
    if ((st = streams_check(planes, n_types, items, n_items, fluct, n_streams))) return st;
    if (!bytes) return LAR_EINVAL;
    *bytes = streams_slice(planes, n_types, items, n_items, fluct) * (size_t)n_streams;
    return LAR_OK;
}

int lar_sim_streams(const lar_plane* planes, int32_t n_types, const float* const* resp, const lar_depos* depos,
                    float nsigma, const lar_fluct* fluct, const lar_batch_item* items, int32_t n_items,
                    float* wave, void* const* streams, int32_t n_streams, void* ws, size_t ws_bytes,
                    void* stream) {
    int st;
    if ((st = streams_check(planes, n_types, items, n_items, fluct, n_streams))) return st;
    if (!resp || !depos || !wave || !streams || !(nsigma > 0.f) || !isfinite(nsigma)) return LAR_EINVAL;
    for (int i = 0; i < n_streams; ++i)
        if (!streams[i] || streams[i] == stream) return LAR_EINVAL;
    for (int i = 0; i < n_items; ++i) {
        if (!resp[items[i].plane_type]) return LAR_EINVAL;
        if (items[i].depo_offset + items[i].n_depos > depos->n) return LAR_EINVAL;
    }
    if (depos->n > 0 && (!depos->q || !depos->t || !depos->x || !depos->sigma_t || !depos->sigma_x))
        return LAR_EINVAL;
    const size_t slice = streams_slice(planes, n_types, items, n_items, fluct);
    if (!ws || ws_bytes < slice * (size_t)n_streams || reinterpret_cast<uintptr_t>(ws) % 256)
        return LAR_EWORKSPACE;
    if (n_items == 0) return LAR_OK;
    hipEvent_t* ev = nullptr;
    if ((st = stream_events(n_streams + 1, &ev))) return st;
    hipStream_t main = (hipStream_t)stream;
    // fork: every worker stream starts after the work already on `stream`
    LAR_TRY(hipEventRecord(ev[0], main));
    const int used = n_items < n_streams ? n_items : n_streams;
    for (int i = 0; i < used; ++i) LAR_TRY(hipStreamWaitEvent((hipStream_t)streams[i], ev[0], 0));
    for (int i = 0; i < n_items; ++i) {
        const lar_batch_item& it = items[i];
        const int si = i % n_streams;
        lar_depos d;
        d.n = it.n_depos;
        d.q = depos->q + it.depo_offset;
        d.t = depos->t + it.depo_offset;
        d.x = depos->x + it.depo_offset;
        d.sigma_t = depos->sigma_t + it.depo_offset;
        d.sigma_x = depos->sigma_x + it.depo_offset;
        lar_fluct f{};
        if (fluct) {
            f = *fluct;
            f.event = it.event;
            f.plane = it.plane;
        }
        if ((st = sim_plane_impl(&planes[it.plane_type], &d, nsigma, fluct ? &f : nullptr, resp[it.plane_type],
                                 wave + it.wave_offset, reinterpret_cast<char*>(ws) + slice * si, slice,
                                 (hipStream_t)streams[si])))
            return st;
    }
    // join: `stream` continues after every worker stream's work
    for (int i = 0; i < used; ++i) {
        LAR_TRY(hipEventRecord(ev[1 + i], (hipStream_t)streams[i]));
        LAR_TRY(hipStreamWaitEvent(main, ev[1 + i], 0));
    }
    return LAR_OK;
}

// fftconv backward workspace: [FT of wave_grad rows: N_w x ld][grid rows: R_rows x ld]
static size_t fftconv_bwd_bytes(const lar_plane* p) {
    size_t ld = (size_t)spec_ld(p);
    return align_up((size_t)p->n_wires * ld * sizeof(float2), 256) +
           align_up((size_t)p->n_wires * p->n_imp * ld * sizeof(float2), 256);
}

int lar_fftconv_backward_workspace(const lar_plane* plane, size_t* bytes) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (!bytes) return LAR_EINVAL;
    *bytes = fftconv_bwd_bytes(plane);
    return LAR_OK;
}

int lar_fftconv_backward(const lar_plane* p, const float* grid, const float* resp,
                         const float* wave_grad, float* grid_grad, float* resp_grad, void* ws,
                         size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_fft(p))) return st;
    if (!resp || !wave_grad || (resp_grad && !grid)) return LAR_EINVAL;
    if (!grid_grad && !resp_grad) return LAR_OK;
    if (!ws || ws_bytes < fftconv_bwd_bytes(p) || reinterpret_cast<uintptr_t>(ws) % 256)
        return LAR_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t ld = spec_ld(p);
    const int rows = p->n_wires * p->n_imp;
    float2* Gt = reinterpret_cast<float2*>(ws);
    float2* Sb = reinterpret_cast<float2*>(reinterpret_cast<char*>(ws) +
                                           align_up((size_t)p->n_wires * ld * sizeof(float2), 256));
    const float scale = (float)(1.0 / ((double)p->nw_fft * (double)p->nt_fft));
    const Sched sc = sched_of(p);
    LAR_TRY(launch_r2c_rows(wave_grad, p->n_ticks, p->n_ticks, p->n_wires, p->nt_fft, Gt, ld, s,
                            sc.row_threads, sc.row_order));
    if (resp_grad)
        LAR_TRY(launch_r2c_rows(grid, p->n_ticks, p->n_ticks, rows, p->nt_fft, Sb, ld, s,
                                sc.row_threads, sc.row_order));
    LAR_TRY(launch_wire_adjoint(Gt, ld, Sb, ld, Sb, ld, p->n_wires, p->n_imp, p->nw_fft, p->nt_fft,
                                reinterpret_cast<const float2*>(resp),
                                reinterpret_cast<float2*>(resp_grad), grid_grad != nullptr, scale, s));
    if (grid_grad)
        LAR_TRY(launch_c2r_rows(Sb, ld, rows, p->nt_fft, grid_grad, p->n_ticks, p->n_ticks, scale, s,
                                nullptr, false, sc.row_threads, sc.row_order));
    return LAR_OK;
}

// backward from a kept grid spectrum: workspace = the FT of wave_grad only
// backward from a kept grid spectrum: FT of the waveform gradient, then the
// grid-gradient spectrum (the kept spectrum is only read)
static size_t fftconv_bwd_spec_bytes(const lar_plane* p) {
    const size_t ld = (size_t)spec_ld(p);
    return align_up((size_t)p->n_wires * ld * sizeof(float2), 256) +
           align_up((size_t)p->n_wires * p->n_imp * ld * sizeof(float2), 256);
}

int lar_fftconv_backward_spec_workspace(const lar_plane* plane, size_t* bytes) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (!bytes) return LAR_EINVAL;
    *bytes = fftconv_bwd_spec_bytes(plane);
    return LAR_OK;
}

int lar_fftconv_backward_spec(const lar_plane* p, const void* grid_spec, const float* resp,
                              const float* wave_grad, float* grid_grad, float* resp_grad,
                              int32_t resp_accumulate, void* ws, size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_fft(p))) return st;
    if (!resp || !wave_grad) return LAR_EINVAL;
    if (!grid_grad && !resp_grad) return LAR_OK;
    if (!grid_spec) return LAR_EINVAL;
    if (!ws || ws_bytes < fftconv_bwd_spec_bytes(p) || reinterpret_cast<uintptr_t>(ws) % 256)
        return LAR_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t ld = spec_ld(p);
    const int rows = p->n_wires * p->n_imp;
    float2* Gt = reinterpret_cast<float2*>(ws);
    float2* Ob = reinterpret_cast<float2*>(reinterpret_cast<char*>(ws) +
                                           align_up((size_t)p->n_wires * ld * sizeof(float2), 256));
    const float2* Sb = reinterpret_cast<const float2*>(grid_spec);
    const float scale = (float)(1.0 / ((double)p->nw_fft * (double)p->nt_fft));
    const Sched sc = sched_of(p);
    LAR_TRY(launch_r2c_rows(wave_grad, p->n_ticks, p->n_ticks, p->n_wires, p->nt_fft, Gt, ld, s,
                            sc.row_threads, sc.row_order));
    LAR_TRY(launch_wire_adjoint(Gt, ld, Sb, ld, Ob, ld, p->n_wires, p->n_imp, p->nw_fft, p->nt_fft,
                                reinterpret_cast<const float2*>(resp),
                                reinterpret_cast<float2*>(resp_grad), grid_grad != nullptr, scale, s,
                                resp_accumulate != 0));
    if (grid_grad)
        LAR_TRY(launch_c2r_rows(Ob, ld, rows, p->nt_fft, grid_grad, p->n_ticks, p->n_ticks, scale, s,
                                nullptr, false, sc.row_threads, sc.row_order));
    return LAR_OK;
}

int lar_raster_backward(const lar_plane* plane, const lar_depos* depos, float nsigma,
                        const float* grid_grad, float* dq, float* dt, float* dx, float* dsigma_t,
                        float* dsigma_x, void* stream) {
    int st;
    if ((st = check_plane(plane))) return st;
    if ((st = check_depos(depos))) return st;
    if (!(nsigma > 0.f) || !isfinite(nsigma)) return LAR_EINVAL;
    if (depos->n == 0) return LAR_OK;
    if (!grid_grad || !dq || !dt || !dx || !dsigma_t || !dsigma_x) return LAR_EINVAL;
    RasterArgs a;
    a.n_ticks = plane->n_ticks;
    a.n_rows = plane->n_wires * plane->n_imp;
    a.ld = plane->n_ticks;
    a.org_t = (double)plane->t0;
    a.wd_t = (double)plane->tick;
    a.org_x = (double)plane->x0 - (double)plane->pitch / 2.0;
    a.wd_x = (double)plane->pitch / (double)plane->n_imp;
    a.nsig = (double)nsigma;
    a.mode = 0;
    a.event = a.plane = 0u;
    a.seed = 0ull;
    LAR_TRY(launch_raster_bwd(a, depos->q, depos->t, depos->x, depos->sigma_t, depos->sigma_x,
                              depos->n, grid_grad, dq, dt, dx, dsigma_t, dsigma_x, (hipStream_t)stream));
    return LAR_OK;
}

// response spectrum workspace: time spectra of the n_imp*(2H+1) response rows
static size_t respspec_bytes(const lar_plane* p, int half_w) {
    return align_up((size_t)p->n_imp * (2 * half_w + 1) * spec_ld(p) * sizeof(float2), 256);
}

int lar_response_spectrum_workspace(const lar_plane* plane, int32_t half_w, int32_t n_rt,
                                    size_t* bytes) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (half_w < 0 || n_rt < 1 || n_rt > plane->nt_fft || !bytes) return LAR_EINVAL;
    *bytes = respspec_bytes(plane, half_w);
    return LAR_OK;
}

int lar_response_spectrum(const lar_plane* plane, const float* r_time, int32_t half_w,
                          int32_t n_rt, float* resp, void* ws, size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (half_w < 0 || n_rt < 1 || n_rt > plane->nt_fft || !r_time || !resp) return LAR_EINVAL;
    if (!ws || ws_bytes < respspec_bytes(plane, half_w) || reinterpret_cast<uintptr_t>(ws) % 256)
        return LAR_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int nrw = 2 * half_w + 1;
    const int64_t ld = spec_ld(plane);
    float2* rows = reinterpret_cast<float2*>(ws);
    LAR_TRY(launch_r2c_rows(r_time, n_rt, n_rt, plane->n_imp * nrw, plane->nt_fft, rows, ld, s));
    LAR_TRY(launch_wire_spectrum(rows, ld, plane->n_imp, nrw, half_w, plane->nw_fft,
                                 plane->nt_fft / 2 + 1, reinterpret_cast<float2*>(resp), s));
    return LAR_OK;
}

int lar_sample_counts(int32_t mode, int64_t n, const float* q, const double* p,
                      const uint32_t* ctr3, uint32_t plane, uint64_t seed, float* out,
                      void* stream) {
    if (mode < 1 || mode > 3 || n < 0 || plane >= 256u) return LAR_EINVAL;
    if (n == 0) return LAR_OK;
    if (!q || !p || !ctr3 || !out) return LAR_EINVAL;
    LAR_TRY(launch_sample_counts(mode, n, q, p, ctr3, plane, seed, out, (hipStream_t)stream));
    return LAR_OK;
}

// ---------------------------------------------------------------- drift, noise, ADC

static int drift_const(const lar_drift_params* prm, const lar_plane_proj* proj, int32_t n_planes,
                       DriftConst& C) {
    if (!prm || n_planes < 0 || n_planes > kDriftMaxPlanes || (n_planes > 0 && !proj)) return LAR_EINVAL;
    if (!(prm->speed > 0.f) || !isfinite(prm->speed) || !(prm->diff_l >= 0.f) || !(prm->diff_t >= 0.f) ||
        !isfinite(prm->diff_l) || !isfinite(prm->diff_t) || !isfinite(prm->lifetime))
        return LAR_EINVAL;
    C.v = (double)prm->speed;
    C.DL = (double)prm->diff_l;
    C.DT = (double)prm->diff_t;
    C.tau = (double)prm->lifetime;
    C.n_planes = n_planes;
    for (int p = 0; p < kDriftMaxPlanes; ++p) {
        const bool on = p < n_planes;
        C.proj[p][0] = on ? (double)proj[p].cos_a : 0.0;
        C.proj[p][1] = on ? (double)proj[p].sin_a : 0.0;
        C.proj[p][2] = on ? (double)proj[p].offset : 0.0;
    }
    return LAR_OK;
}

int lar_drift(const lar_drift_params* prm, const float* q0, const float* t0, const float* xd,
              const float* y, const float* z, int64_t n, const lar_plane_proj* proj, int32_t n_planes,
              float* q, float* t, float* sigma_t, float* sigma_x, float* x, void* stream) {
    DriftConst C;
    int st;
    if ((st = drift_const(prm, proj, n_planes, C))) return st;
    if (n < 0) return LAR_EINVAL;
    if (n == 0) return LAR_OK;
    if (!q0 || !t0 || !xd || !y || !z || !q || !t || !sigma_t || !sigma_x || (n_planes > 0 && !x))
        return LAR_EINVAL;
    LAR_TRY(launch_drift(C, q0, t0, xd, y, z, n, q, t, sigma_t, sigma_x, x, (hipStream_t)stream));
    return LAR_OK;
}

int lar_drift_backward_workspace(int64_t n, size_t* bytes) {
    if (n < 0 || !bytes) return LAR_EINVAL;
    *bytes = (size_t)kDriftMaxBlocks * 4 * sizeof(double);
    return LAR_OK;
}

int lar_drift_backward(const lar_drift_params* prm, const float* q0, const float* xd, int64_t n,
                       const lar_plane_proj* proj, int32_t n_planes, const float* gq, const float* gt,
                       const float* gsigma_t, const float* gsigma_x, const float* gx, float* dq0,
                       float* dt0, float* dxd, float* dy, float* dz, float* dparams, void* ws,
                       size_t ws_bytes, void* stream) {
    DriftConst C;
    int st;
    if ((st = drift_const(prm, proj, n_planes, C))) return st;
    if (n < 0) return LAR_EINVAL;
    if (dparams && (!ws || ws_bytes < (size_t)kDriftMaxBlocks * 4 * sizeof(double) ||
                    reinterpret_cast<uintptr_t>(ws) % 256))
        return LAR_EWORKSPACE;
    if (n > 0 && (!q0 || !xd || !gq || !gt || !gsigma_t || !gsigma_x || (n_planes > 0 && !gx)))
        return LAR_EINVAL;
    LAR_TRY(launch_drift_bwd(C, q0, xd, n, gq, gt, gsigma_t, gsigma_x, gx, dq0, dt0, dxd, dy, dz, dparams,
                             reinterpret_cast<double*>(ws), (hipStream_t)stream));
    return LAR_OK;
}

// noise workspace: the random half spectra [n_wires][ld]
static size_t noise_bytes(const lar_plane* p) {
    return align_up((size_t)p->n_wires * (size_t)spec_ld(p) * sizeof(float2), 256);
}

int lar_noise_workspace(const lar_plane* plane, size_t* bytes) {
    int st;
    if ((st = check_fft(plane))) return st;
    if (!bytes) return LAR_EINVAL;
    *bytes = noise_bytes(plane);
    return LAR_OK;
}

int lar_noise(const lar_plane* p, const float* amp, uint64_t seed, uint32_t event, uint32_t plane_id,
              float* noise, void* ws, size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_fft(p))) return st;
    if (!amp || !noise || plane_id >= 256u) return LAR_EINVAL;
    if (!ws || ws_bytes < noise_bytes(p) || reinterpret_cast<uintptr_t>(ws) % 256) return LAR_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t ld = spec_ld(p);
    float2* X = reinterpret_cast<float2*>(ws);
    const Sched sc = sched_of(p);
    LAR_TRY(launch_noise_spectrum(amp, p->nt_fft / 2 + 1, p->n_wires, seed, event, plane_id, X, ld, s));
    LAR_TRY(launch_c2r_rows(X, ld, p->n_wires, p->nt_fft, noise, p->n_ticks, p->n_ticks,
                            (float)(1.0 / (double)p->nt_fft), s, nullptr, false, sc.row_threads,
                            sc.row_order));
    return LAR_OK;
}

int lar_digitize(const float* wave, const float* noise, int64_t n, float gain, float baseline, int32_t bits,
                 uint16_t* adc, void* stream) {
    if (n < 0 || bits < 1 || bits > 16 || !isfinite(gain) || !isfinite(baseline)) return LAR_EINVAL;
    if (n == 0) return LAR_OK;
    if (!wave || !adc) return LAR_EINVAL;
    LAR_TRY(launch_digitize(wave, noise, n, gain, baseline, bits, adc, (hipStream_t)stream));
    return LAR_OK;
}

}  // extern "C"
