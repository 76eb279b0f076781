// batch.hip -- many (event, plane) items in one launch sequence, captured
// once into a hipGraph and replayed (the paper raises throughput by running
// independent processes per GPU, Sec. 3.3; here one process runs them as
// batched launches sharing each plane type's response).
//
// Items are grouped by plane type and each type's items are cut into waves
// of at most K items, K as large as the caller's workspace allows.  One wave
// holds K grids, K time spectra and K wire-pass outputs in an arena that
// every wave of every type reuses, so memory is bounded by K, not by the
// number of items.  Per wave: clear the grids, one raster launch over the
// wave's items (a table of them, built on the device each run by a
// segmented prefix sum of their sub-chunk counts), one launch per FFT stage
// over the wave's rows; the wire pass runs the blocks of one tile for every
// item of the wave together on one XCD, so the tile's response slabs come
// from that XCD's L2.
//
// With more than one wave the grids are double-buffered (waves alternate
// between two grid regions) and the FFT stages of each wave run on a second
// stream: wave w's memory-bound transforms overlap wave w+1's ALU-bound
// raster.  The raster of wave w+2 waits for wave w's time R2C (the last
// reader of its grid region); the FFT stages of successive waves, which
// share the spectrum regions, stay in order on their stream.  A run forks
// the second stream from the caller's and joins it back at the end.
//
// Workspace layout (all 256-byte aligned):
//   item records in wave order | raster item table | wave-local sub-chunk
//   prefix | per-type plane constants | output row offsets | arena (grid,
//   spectrum and wire-output regions, each sized for the largest wave) |
//   second grid region (more than one wave) | raster queue
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <functional>
#include <new>
#include <vector>

#include "lar_internal.hpp"

using namespace lar;

namespace {

size_t al(size_t v) { return (v + 255) / 256 * 256; }

int64_t spec_ld_of(const lar_plane& p) { return ((int64_t)(p.nt_fft / 2 + 1) + 15) / 16 * 16; }

bool smooth(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

bool plane_ok(const lar_plane& p) {
    if (p.n_wires < 1 || p.n_imp < 1 || p.n_ticks < 1) return false;
    if (!(p.tick > 0.f) || !(p.pitch > 0.f) || !isfinite(p.x0) || !isfinite(p.t0)) return false;
    if ((int64_t)p.n_wires * p.n_imp > INT_MAX / 2) return false;
    if (p.nt_fft % 2 || !smooth(p.nt_fft / 2) || p.nt_fft < p.n_ticks || p.nt_fft > 16384) return false;
    if (!smooth(p.nw_fft) || p.nw_fft < p.n_wires || p.nw_fft > 1024) return false;
    return true;
}

// Per-item record on the device (wave order).
struct DevItem {
    int32_t type, slot;         // plane type, position within its wave
    uint32_t event, plane;
    int64_t depo_offset, n_depos;
    int32_t wave_first;         // index (wave order) of the first item of its wave
    int32_t buf;                // grid region of its wave: 0 (the arena) or 1
};

// Per-type constants the table kernel needs.
struct DevType {
    RasterArgs proto;           // geometry and fluctuation; event and plane set per item
    int64_t grid_stride;        // floats between the grids of consecutive slots
    float* grid0;               // grid of slot 0 in the arena
    float* grid1;               // grid of slot 0 in the second grid region
};

struct Wave {
    int type, first, count;     // items [first, first + count) in wave order
    int64_t n_depos, total_sub;
};

struct Layout {
    size_t items, table, prefix, types, rowoff, arena, grid1, raster, total;
    int K = 0;                                  // items per wave
    std::vector<int> order;                     // wave order -> item index
    std::vector<Wave> waves;
    std::vector<size_t> gsz, ssz, msz;          // per type, per slot
    size_t arena_bytes = 0, grid1_bytes = 0, raster_bytes = 0;
    size_t s_off = 0, m_off = 0;                // spectra and wire outputs within the arena
    int64_t total_rows_out = 0;
};

size_t raster_ws_for(const lar_fluct* f, int64_t sub, int64_t depos) {
    if (!f || f->mode == 0 || sub <= 0) return 0;
    size_t b = raster_ws_fixed_subs(sub);
    if (f->mode != 3) b += al(((size_t)depos * 48 + 4096) * kDeferredBytes);
    return b;
}

int check_items(const lar_plane* planes, int n_types, const lar_batch_item* items, int n_items,
                const lar_fluct* fluct) {
    if (!planes || n_types < 1 || !items || n_items < 1) return LAR_EINVAL;
    if (n_items >= (1 << 27)) return LAR_ESIZE;   // item index shares a 32-bit word with queue marks
    if (fluct && (fluct->mode < 0 || fluct->mode > 3 || fluct->plane >= 256u)) return LAR_EINVAL;
    for (int t = 0; t < n_types; ++t) {
        if (!plane_ok(planes[t])) return LAR_ESIZE;
        // a drawn bin's counter word is m * n_ticks + j
        if (fluct && fluct->mode != 0 &&
            (int64_t)planes[t].n_wires * planes[t].n_imp * planes[t].n_ticks > (int64_t)UINT32_MAX)
            return LAR_ESIZE;
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

// Layout for waves of at most K items per type (K >= 1).
void layout(const lar_plane* planes, int n_types, const lar_batch_item* items, int n_items,
            const lar_fluct* fluct, int K, Layout& L) {
    L.K = K;
    L.order.clear();
    L.waves.clear();
    L.gsz.assign(n_types, 0);
    L.ssz.assign(n_types, 0);
    L.msz.assign(n_types, 0);
    L.arena_bytes = 0;
    L.grid1_bytes = 0;
    L.raster_bytes = 0;
    L.total_rows_out = 0;
    size_t grids_max = 0, specs_max = 0, outs_max = 0;
    int64_t max_sub = 0, max_depos = 0;
    for (int t = 0; t < n_types; ++t) {
        const lar_plane& p = planes[t];
        L.gsz[t] = al((size_t)p.n_wires * p.n_imp * p.n_ticks * sizeof(float));
        L.ssz[t] = al((size_t)p.n_wires * p.n_imp * spec_ld_of(p) * sizeof(float2));
        L.msz[t] = al((size_t)p.n_wires * spec_ld_of(p) * sizeof(float2));
        std::vector<int> mine;
        for (int i = 0; i < n_items; ++i)
            if (items[i].plane_type == t) mine.push_back(i);
        for (size_t a = 0; a < mine.size(); a += (size_t)K) {
            Wave w;
            w.type = t;
            w.first = (int)L.order.size();
            w.count = (int)std::min<size_t>((size_t)K, mine.size() - a);
            w.n_depos = 0;
            w.total_sub = 0;
            for (int j = 0; j < w.count; ++j) {
                const lar_batch_item& it = items[mine[a + j]];
                L.order.push_back(mine[a + j]);
                w.n_depos += it.n_depos;
                w.total_sub += raster_subchunks(it.n_depos);
                L.total_rows_out += p.n_wires;
            }
            max_sub = std::max(max_sub, w.total_sub);
            max_depos = std::max(max_depos, w.n_depos);
            grids_max = std::max(grids_max, L.gsz[t] * (size_t)w.count);
            specs_max = std::max(specs_max, L.ssz[t] * (size_t)w.count);
            outs_max = std::max(outs_max, L.msz[t] * (size_t)w.count);
            L.waves.push_back(w);
        }
    }
    // the arena's grid, spectrum and output regions are disjoint and sized for
    // the largest wave: a wave's grids never overlap the spectra or outputs
    // that an earlier wave's FFT stages may still be using on the FFT stream
    L.s_off = grids_max;
    L.m_off = grids_max + specs_max;
    L.arena_bytes = grids_max + specs_max + outs_max;
    if (L.waves.size() > 1) L.grid1_bytes = grids_max;   // double-buffered grids
    L.raster_bytes = raster_ws_for(fluct, max_sub, max_depos);
    size_t off = 0;
    L.items = off;  off += al(sizeof(DevItem) * (size_t)n_items);
    L.table = off;  off += al(sizeof(RasterItem) * (size_t)n_items);
    L.prefix = off; off += al(sizeof(int64_t) * (size_t)n_items);
    L.types = off;  off += al(sizeof(DevType) * (size_t)n_types);
    L.rowoff = off; off += al(sizeof(int64_t) * (size_t)L.total_rows_out);
    L.arena = off;  off += L.arena_bytes;
    L.grid1 = off;  off += L.grid1_bytes;
    L.raster = off; off += L.raster_bytes;
    L.total = off;
}

int max_type_count(const lar_batch_item* items, int n_items, int n_types) {
    std::vector<int> c(n_types, 0);
    int m = 0;
    for (int i = 0; i < n_items; ++i) m = std::max(m, ++c[items[i].plane_type]);
    return m;
}

// ---- device table of the raster items: one workgroup, a prefix sum of the
// items' sub-chunk counts in wave order, restarted at each wave
constexpr int kTableThreads = 1024;

__global__ __launch_bounds__(kTableThreads) void k_batch_table(const DevItem* __restrict__ it,
                                                                const DevType* __restrict__ ty, int n_items,
                                                                lar_depos depos, RasterItem* __restrict__ out,
                                                                int64_t* __restrict__ prefix) {
    __shared__ int64_t s_scan[kTableThreads];
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    // global exclusive prefix of the sub-chunk counts
    for (int c0 = 0; c0 < n_items; c0 += kTableThreads) {
        const int i = c0 + (int)threadIdx.x;
        const int64_t v = i < n_items ? raster_subchunks(it[i].n_depos) : 0;
        s_scan[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kTableThreads; o <<= 1) {   // Hillis-Steele inclusive scan
            const int64_t a = threadIdx.x >= (unsigned)o ? s_scan[threadIdx.x - o] : 0;
            __syncthreads();
            s_scan[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < n_items) prefix[i] = s_carry + s_scan[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kTableThreads - 1) s_carry += s_scan[kTableThreads - 1];
        __syncthreads();
    }
    // every prefix is written; each item's wave-local start, and its record
    for (int i = threadIdx.x; i < n_items; i += kTableThreads) {
        const DevItem d = it[i];
        const DevType& T = ty[d.type];
        RasterItem r;
        r.A = T.proto;
        r.A.event = d.event;
        r.A.plane = d.plane;
        r.q = depos.q + d.depo_offset;
        r.t = depos.t + d.depo_offset;
        r.x = depos.x + d.depo_offset;
        r.st = depos.sigma_t + d.depo_offset;
        r.sx = depos.sigma_x + d.depo_offset;
        r.grid = (d.buf ? T.grid1 : T.grid0) + (int64_t)d.slot * T.grid_stride;
        r.n = d.n_depos;
        r.sub_begin = prefix[i] - prefix[d.wave_first];
        out[i] = r;
    }
}

}  // namespace

struct lar_batch {
    // each step enqueues on the main stream or on the FFT stream
    std::vector<std::function<hipError_t(hipStream_t, hipStream_t)>> steps;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // second stream of an eager run (default priority) and the events that
    // order the two streams: fork, join, raster done, time R2C done (by
    // wave parity)
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_rast = nullptr, ev_r2c[2] = {nullptr, nullptr};
    // for the backward pass (mean path only)
    int mode = 0;
    std::vector<lar_plane> planes;
    std::vector<const float*> resp;
    std::vector<lar_batch_item> items;   // wave order
    std::vector<Wave> waves;
    std::vector<RasterArgs> proto;       // per type
    lar_depos depos{};
    char* arena = nullptr;
    char* grid1 = nullptr;               // second grid region (more than one wave), else null
    const RasterItem* dtab = nullptr;
    const int64_t* drow = nullptr;
    const DevItem* ditp = nullptr;
    const DevType* dtyp = nullptr;
    int64_t* dpre = nullptr;
    bool rows_even = false;
    // wave whose time spectra the arena still holds (the last wave of the
    // last run), -1 when none: the backward pass reuses them
    int kept_wave = -1;
    std::vector<int64_t> row0;           // per wave: first output row in drow
    std::vector<size_t> gsz, ssz, msz;
    size_t s_off = 0, m_off = 0;         // spectrum and output regions within the arena
};

namespace {

RasterArgs args_of(const lar_plane& p, float nsigma, const lar_fluct* fluct) {
    RasterArgs a;
    a.n_ticks = p.n_ticks;
    a.n_rows = p.n_wires * p.n_imp;
    a.ld = p.n_ticks;
    a.org_t = (double)p.t0;
    a.wd_t = (double)p.tick;
    a.org_x = (double)p.x0 - (double)p.pitch / 2.0;
    a.wd_x = (double)p.pitch / (double)p.n_imp;
    a.nsig = (double)nsigma;
    a.mode = fluct ? fluct->mode : 0;
    a.event = a.plane = 0u;
    a.seed = fluct ? fluct->seed : 0ull;
    return a;
}

// Largest wave size whose layout fits in ws_bytes (0 if none does).  Every
// type in one wave is tried first: below that size the largest type takes
// two waves or more, the layout holds the second grid region, and its size
// grows with the wave size, so the rest is a bisection.
int fit_waves(const lar_plane* planes, int n_types, const lar_batch_item* items, int n_items,
              const lar_fluct* fluct, size_t ws_bytes, Layout& L) {
    const int m = max_type_count(items, n_items, n_types);
    layout(planes, n_types, items, n_items, fluct, m, L);
    if (L.total <= ws_bytes) return m;
    int lo = 1, hi = m - 1, best = 0;
    while (lo <= hi) {
        const int mid = lo + (hi - lo) / 2;
        layout(planes, n_types, items, n_items, fluct, mid, L);
        if (L.total <= ws_bytes) {
            best = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    if (best) layout(planes, n_types, items, n_items, fluct, best, L);
    return best;
}

// Frees a plan and the HIP objects it owns (any of them may be null).
void release(lar_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : {b->ev_fork, b->ev_join, b->ev_rast, b->ev_r2c[0], b->ev_r2c[1]})
        if (e) (void)hipEventDestroy(e);
    if (b->s2) (void)hipStreamDestroy(b->s2);
    delete b;
}

// fork: s2 waits for what s has enqueued so far; join: s waits for s2.
hipError_t fork_join(lar_batch* b, hipStream_t s, hipStream_t s2, bool fork) {
    hipEvent_t e = fork ? b->ev_fork : b->ev_join;
    hipError_t r = hipEventRecord(e, fork ? s : s2);
    return r == hipSuccess ? hipStreamWaitEvent(fork ? s2 : s, e, 0) : r;
}

}  // namespace

extern "C" {

int lar_batch_workspace_waves(const lar_plane* planes, int32_t n_types, const lar_batch_item* items,
                              int32_t n_items, const lar_fluct* fluct, int32_t max_wave, size_t* bytes) {
    if (!bytes || max_wave < 0) return LAR_EINVAL;
    int st = check_items(planes, n_types, items, n_items, fluct);
    if (st) return st;
    const int m = max_type_count(items, n_items, n_types);
    Layout L;
    layout(planes, n_types, items, n_items, fluct, max_wave == 0 ? m : std::min(max_wave, m), L);
    *bytes = L.total;
    return LAR_OK;
}

int lar_batch_workspace(const lar_plane* planes, int32_t n_types, const lar_batch_item* items,
                        int32_t n_items, const lar_fluct* fluct, size_t* bytes) {
    return lar_batch_workspace_waves(planes, n_types, items, n_items, fluct, 0, bytes);
}

int lar_batch_create(const lar_plane* planes, int32_t n_types, const float* const* resp,
                     const lar_depos* depos, float nsigma, const lar_fluct* fluct,
                     const lar_batch_item* items, int32_t n_items, float* wave, void* ws,
                     size_t ws_bytes, int32_t use_graph, lar_batch** out) {
    if (!out || !resp || !depos || !wave || !(nsigma > 0.f) || !isfinite(nsigma)) return LAR_EINVAL;
    *out = nullptr;
    int st = check_items(planes, n_types, items, n_items, fluct);
    if (st) return st;
    std::vector<int> count(n_types, 0);
    for (int i = 0; i < n_items; ++i) count[items[i].plane_type]++;
    for (int t = 0; t < n_types; ++t)
        if (count[t] && !resp[t]) return LAR_EINVAL;
    int64_t total_depos = 0;
    for (int i = 0; i < n_items; ++i)
        total_depos = std::max(total_depos, items[i].depo_offset + items[i].n_depos);
    if (total_depos > depos->n) return LAR_EINVAL;
    if (depos->n > 0 && (!depos->q || !depos->t || !depos->x || !depos->sigma_t || !depos->sigma_x))
        return LAR_EINVAL;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return LAR_EWORKSPACE;
    Layout L;
    if (!fit_waves(planes, n_types, items, n_items, fluct, ws_bytes, L)) return LAR_EWORKSPACE;
    char* W = reinterpret_cast<char*>(ws);
    const int mode = fluct ? fluct->mode : 0;

    // ---- host tables, uploaded once
    std::vector<DevItem> dit(n_items);
    std::vector<DevType> dty(n_types);
    for (int t = 0; t < n_types; ++t) {
        dty[t].proto = args_of(planes[t], nsigma, fluct);
        dty[t].grid_stride = (int64_t)(L.gsz[t] / sizeof(float));
        dty[t].grid0 = reinterpret_cast<float*>(W + L.arena);
        dty[t].grid1 = reinterpret_cast<float*>(W + (L.grid1_bytes ? L.grid1 : L.arena));
    }
    std::vector<int64_t> rowoff;
    rowoff.reserve(L.total_rows_out);
    std::vector<int64_t> row0;
    bool even = true;
    for (size_t wi = 0; wi < L.waves.size(); ++wi) {
        const Wave& w = L.waves[wi];
        row0.push_back((int64_t)rowoff.size());
        for (int j = 0; j < w.count; ++j) {
            const int i = w.first + j;
            const lar_batch_item& it = items[L.order[i]];
            DevItem& d = dit[i];
            d.type = it.plane_type;
            d.slot = j;
            d.event = it.event;
            d.plane = it.plane;
            d.depo_offset = it.depo_offset;
            d.n_depos = it.n_depos;
            d.wave_first = w.first;
            d.buf = (L.grid1_bytes && (wi % 2)) ? 1 : 0;
            const lar_plane& p = planes[it.plane_type];
            for (int r = 0; r < p.n_wires; ++r) {
                const int64_t o = it.wave_offset + (int64_t)r * p.n_ticks;
                rowoff.push_back(o);
                if (o % 2) even = false;
            }
        }
    }
    if (hipMemcpy(W + L.items, dit.data(), sizeof(DevItem) * n_items, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(W + L.types, dty.data(), sizeof(DevType) * n_types, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(W + L.rowoff, rowoff.data(), sizeof(int64_t) * rowoff.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
        return LAR_EHIP;

    lar_batch* b = new (std::nothrow) lar_batch;
    if (!b) return LAR_EINVAL;
    b->mode = mode;
    b->planes.assign(planes, planes + n_types);
    b->resp.assign(resp, resp + n_types);
    for (int i = 0; i < n_items; ++i) b->items.push_back(items[L.order[i]]);
    b->waves = L.waves;
    for (int t = 0; t < n_types; ++t) b->proto.push_back(dty[t].proto);
    b->depos = *depos;
    b->arena = W + L.arena;
    b->grid1 = L.grid1_bytes ? W + L.grid1 : nullptr;
    b->dtab = reinterpret_cast<const RasterItem*>(W + L.table);
    b->drow = reinterpret_cast<const int64_t*>(W + L.rowoff);
    b->row0 = row0;
    b->rows_even = even;
    b->ditp = reinterpret_cast<const DevItem*>(W + L.items);
    b->dtyp = reinterpret_cast<const DevType*>(W + L.types);
    b->dpre = reinterpret_cast<int64_t*>(W + L.prefix);
    b->gsz = L.gsz;
    b->ssz = L.ssz;
    b->msz = L.msz;
    b->s_off = L.s_off;
    b->m_off = L.m_off;
    if (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_rast, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_r2c[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_r2c[1], hipEventDisableTiming) != hipSuccess ||
        (!use_graph && hipStreamCreateWithFlags(&b->s2, hipStreamNonBlocking) != hipSuccess)) {
        release(b);
        return LAR_EHIP;
    }

    // ---- the launch sequence: the main stream s clears the grids and runs
    // the rasters, the FFT stream s2 the transforms
    const DevItem* ditp = reinterpret_cast<const DevItem*>(W + L.items);
    const DevType* dtyp = reinterpret_cast<const DevType*>(W + L.types);
    RasterItem* dtab = reinterpret_cast<RasterItem*>(W + L.table);
    int64_t* dpre = reinterpret_cast<int64_t*>(W + L.prefix);
    const lar_depos dep = *depos;
    b->steps.push_back([=](hipStream_t s, hipStream_t) {
        hipLaunchKernelGGL(k_batch_table, dim3(1), dim3(kTableThreads), 0, s, ditp, dtyp, n_items, dep, dtab,
                           dpre);
        return hipGetLastError();
    });
    const bool dbl = L.grid1_bytes > 0;
    const hipEvent_t ev_rast = b->ev_rast;
    void* rws = W + L.raster;
    const size_t rws_bytes = L.raster_bytes;
    for (size_t wi = 0; wi < L.waves.size(); ++wi) {
        const Wave w = L.waves[wi];
        const int t = w.type, k = w.count;
        const lar_plane p = planes[t];
        const int64_t ld = spec_ld_of(p);
        const int rows = p.n_wires * p.n_imp;
        float* g = reinterpret_cast<float*>(W + ((dbl && (wi % 2)) ? L.grid1 : L.arena));
        const hipEvent_t ev_r2c = b->ev_r2c[wi % 2];
        float2* S = reinterpret_cast<float2*>(W + L.arena + L.s_off);
        float2* M = reinterpret_cast<float2*>(W + L.arena + L.m_off);
        const int64_t gstride = (int64_t)(L.gsz[t] / sizeof(float));
        const int64_t sstride = (int64_t)(L.ssz[t] / sizeof(float2));
        const int64_t mstride = (int64_t)(L.msz[t] / sizeof(float2));
        const float2* R = reinterpret_cast<const float2*>(resp[t]);
        const int F = p.nt_fft / 2 + 1;
        const float scale = (float)(1.0 / ((double)p.nw_fft * (double)p.nt_fft));
        const int64_t* ro = b->drow + row0[wi];
        const Sched sc = sched_for(p.n_wires, p.n_imp, p.n_ticks, p.nt_fft, p.nw_fft);
        const RasterItem* wtab = dtab + w.first;
        const RasterItem one{};
        // this grid region was last read by the time R2C of wave wi - 2
        if (dbl && wi >= 2)
            b->steps.push_back([=](hipStream_t s, hipStream_t) { return hipStreamWaitEvent(s, ev_r2c, 0); });
        b->steps.push_back([=](hipStream_t s, hipStream_t) { return launch_fill(g, gstride * k, s); });
        if (w.total_sub > 0)
            b->steps.push_back([=](hipStream_t s, hipStream_t) {
                return launch_raster_items(mode, one, wtab, k, w.total_sub, rws, rws_bytes, s, nullptr,
                                           sc.raster_tile);
            });
        b->steps.push_back([=](hipStream_t s, hipStream_t s2) {
            hipError_t e = hipEventRecord(ev_rast, s);
            return e == hipSuccess ? hipStreamWaitEvent(s2, ev_rast, 0) : e;
        });
        // grids of a wave are gstride floats apart: one launch when unpadded
        if (gstride == (int64_t)rows * p.n_ticks && sstride == (int64_t)rows * ld) {
            b->steps.push_back([=](hipStream_t, hipStream_t s2) {
                return launch_r2c_rows(g, p.n_ticks, p.n_ticks, rows * k, p.nt_fft, S, ld, s2, sc.row_threads,
                                       sc.row_order);
            });
        } else {
            for (int r = 0; r < k; ++r)
                b->steps.push_back([=](hipStream_t, hipStream_t s2) {
                    return launch_r2c_rows(g + r * gstride, p.n_ticks, p.n_ticks, rows, p.nt_fft, S + r * sstride,
                                           ld, s2, sc.row_threads, sc.row_order);
                });
        }
        if (dbl) b->steps.push_back([=](hipStream_t, hipStream_t s2) { return hipEventRecord(ev_r2c, s2); });
        b->steps.push_back([=](hipStream_t, hipStream_t s2) {
            return launch_wire_fused(S, ld, p.n_wires, p.n_imp, p.nw_fft, F, R, M, ld, s2, k, sstride, mstride,
                                     sc.wire_cols, sc.wire_threads, sc.wire_order);
        });
        if (mstride == (int64_t)p.n_wires * ld) {
            b->steps.push_back([=](hipStream_t, hipStream_t s2) {
                return launch_c2r_rows(M, ld, p.n_wires * k, p.nt_fft, wave, p.n_ticks, p.n_ticks, scale, s2, ro,
                                       even, sc.row_threads, sc.row_order);
            });
        } else {
            for (int r = 0; r < k; ++r)
                b->steps.push_back([=](hipStream_t, hipStream_t s2) {
                    return launch_c2r_rows(M + r * mstride, ld, p.n_wires, p.nt_fft, wave, p.n_ticks, p.n_ticks,
                                           scale, s2, ro + (int64_t)r * p.n_wires, even, sc.row_threads,
                                           sc.row_order);
                });
        }
    }
    if (use_graph) {
        hipStream_t cs = nullptr, cs2 = nullptr;
        bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            ok = fork_join(b, cs, cs2, true) == hipSuccess;
            for (auto& f : b->steps) ok = ok && f(cs, cs2) == hipSuccess;
            ok = ok && fork_join(b, cs, cs2, false) == hipSuccess;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &g);
            ok = ok && e == hipSuccess && g;
            if (ok) {
                b->graph = g;
                ok = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess;
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        if (cs2) (void)hipStreamDestroy(cs2);
        if (cs) (void)hipStreamDestroy(cs);
        if (!ok) {
            release(b);
            return LAR_EHIP;
        }
    }
    *out = b;
    return LAR_OK;
}

int lar_batch_waves(const lar_batch* b, int32_t* n_waves, int32_t* max_items) {
    if (!b) return LAR_EINVAL;
    int m = 0;
    for (const Wave& w : b->waves) m = std::max(m, w.count);
    if (n_waves) *n_waves = (int32_t)b->waves.size();
    if (max_items) *max_items = m;
    return LAR_OK;
}

int lar_batch_run(lar_batch* b, void* stream) {
    if (!b) return LAR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    b->kept_wave = -1;
    if (b->exec) {
        hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return ((void)hipGetLastError(), LAR_EHIP);
    } else {
        if (fork_join(b, s, b->s2, true) != hipSuccess) return LAR_EHIP;
        for (auto& f : b->steps)
            if (f(s, b->s2) != hipSuccess) return ((void)fork_join(b, s, b->s2, false), LAR_EHIP);
        if (fork_join(b, s, b->s2, false) != hipSuccess) return LAR_EHIP;
    }
    b->kept_wave = (int)b->waves.size() - 1;
    return LAR_OK;
}

#define LAR_BTRY(expr)                                            \
    do {                                                          \
        if ((expr) != hipSuccess) return ((void)hipGetLastError(), LAR_EHIP); \
    } while (0)

int lar_batch_backward(lar_batch* b, const float* wave_grad, float* const* resp_grad, float* dq, float* dt,
                       float* dx, float* dsigma_t, float* dsigma_x, void* stream) {
    if (!b || !wave_grad) return LAR_EINVAL;
    if (b->mode != 0) return LAR_EINVAL;   // gradients of the mean path only
    const bool want_depo = dq || dt || dx || dsigma_t || dsigma_x;
    if (want_depo && !(dq && dt && dx && dsigma_t && dsigma_x)) return LAR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_batch_table, dim3(1), dim3(kTableThreads), 0, s, b->ditp, b->dtyp, (int)b->items.size(),
                       b->depos, const_cast<RasterItem*>(b->dtab), b->dpre);
    LAR_BTRY(hipGetLastError());
    std::vector<bool> first(b->planes.size(), true);
    // last wave first: right after lar_batch_run its spectra are still in the arena
    const int kept = b->kept_wave;
    b->kept_wave = -1;
    for (int wi = (int)b->waves.size() - 1; wi >= 0; --wi) {
        const Wave& w = b->waves[wi];
        const int t = w.type, k = w.count;
        const lar_plane& p = b->planes[t];
        const int64_t ld = spec_ld_of(p);
        const int rows = p.n_wires * p.n_imp;
        // the grid region this wave's raster items point at
        float* g = reinterpret_cast<float*>((b->grid1 && (wi % 2)) ? b->grid1 : b->arena);
        float2* S = reinterpret_cast<float2*>(b->arena + b->s_off);
        float2* M = reinterpret_cast<float2*>(b->arena + b->m_off);
        const int64_t gstride = (int64_t)(b->gsz[t] / sizeof(float));
        const int64_t sstride = (int64_t)(b->ssz[t] / sizeof(float2));
        const int64_t mstride = (int64_t)(b->msz[t] / sizeof(float2));
        const float scale = (float)(1.0 / ((double)p.nw_fft * (double)p.nt_fft));
        const Sched sc = sched_for(p.n_wires, p.n_imp, p.n_ticks, p.nt_fft, p.nw_fft);
        const int64_t* ro = b->drow + b->row0[wi];
        float2* dR = resp_grad ? reinterpret_cast<float2*>(resp_grad[t]) : nullptr;
        // the wave's grids and their time spectra, recomputed (patches are not
        // stored) unless the forward run left them in the arena
        if (wi != kept) {
            LAR_BTRY(launch_fill(g, gstride * k, s));
            if (w.total_sub > 0) {
                const RasterItem one{};
                LAR_BTRY(launch_raster_items(0, one, b->dtab + w.first, k, w.total_sub, nullptr, 0, s, nullptr,
                                             sc.raster_tile));
            }
            if (gstride == (int64_t)rows * p.n_ticks && sstride == (int64_t)rows * ld) {
                LAR_BTRY(launch_r2c_rows(g, p.n_ticks, p.n_ticks, rows * k, p.nt_fft, S, ld, s, sc.row_threads,
                                         sc.row_order));
            } else {
                for (int r = 0; r < k; ++r)
                    LAR_BTRY(launch_r2c_rows(g + r * gstride, p.n_ticks, p.n_ticks, rows, p.nt_fft, S + r * sstride,
                                             ld, s, sc.row_threads, sc.row_order));
            }
        }
        // time spectra of the waveform gradients, into the wire-pass buffers
        if (mstride == (int64_t)p.n_wires * ld) {
            LAR_BTRY(launch_r2c_rows(wave_grad, p.n_ticks, p.n_ticks, p.n_wires * k, p.nt_fft, M, ld, s,
                                     sc.row_threads, sc.row_order, ro, b->rows_even));
        } else {
            for (int r = 0; r < k; ++r)
                LAR_BTRY(launch_r2c_rows(wave_grad, p.n_ticks, p.n_ticks, p.n_wires, p.nt_fft, M + r * mstride, ld,
                                         s, sc.row_threads, sc.row_order, ro + (int64_t)r * p.n_wires,
                                         b->rows_even));
        }
        // the wave's grids are dead until the grid gradients: scratch for the
        // response-gradient partials of the item groups
        LAR_BTRY(launch_wire_adjoint_items(M, ld, mstride, S, ld, sstride, k, p.n_wires, p.n_imp, p.nw_fft,
                                           p.nt_fft, reinterpret_cast<const float2*>(b->resp[t]), dR, scale, s,
                                           !first[t], g, b->gsz[t] * k));
        first[t] = false;
        if (!want_depo) continue;
        if (gstride == (int64_t)rows * p.n_ticks && sstride == (int64_t)rows * ld) {
            LAR_BTRY(launch_c2r_rows(S, ld, rows * k, p.nt_fft, g, p.n_ticks, p.n_ticks, scale, s, nullptr, false,
                                     sc.row_threads, sc.row_order));
        } else {
            for (int r = 0; r < k; ++r)
                LAR_BTRY(launch_c2r_rows(S + r * sstride, ld, rows, p.nt_fft, g + r * gstride, p.n_ticks, p.n_ticks,
                                         scale, s, nullptr, false, sc.row_threads, sc.row_order));
        }
        for (int j = 0; j < k; ++j) {
            const lar_batch_item& it = b->items[w.first + j];
            if (it.n_depos == 0) continue;
            const int64_t o = it.depo_offset;
            RasterArgs a = b->proto[t];
            const lar_depos& D = b->depos;
            LAR_BTRY(launch_raster_bwd(a, D.q + o, D.t + o, D.x + o, D.sigma_t + o, D.sigma_x + o, it.n_depos,
                                       g + j * gstride, dq + o, dt + o, dx + o, dsigma_t + o, dsigma_x + o, s));
        }
    }
    return LAR_OK;
}

int lar_batch_destroy(lar_batch* b) {
    release(b);
    return LAR_OK;
}

}  // extern "C"
