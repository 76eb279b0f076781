// batch.hip -- many (event, plane) items in one launch sequence, captured
// once into a hipGraph and replayed.
//
// Layout in the caller's workspace (all 256-byte aligned):
//   item table (RasterItem[n_items]) | output row-offset table (int64 per
//   waveform row) | grids, grouped by plane type | time spectra, grouped by
//   plane type | wire-pass outputs, grouped by plane type | raster queue.
// Grouping by plane type makes the rows of one type contiguous, so each
// type's three FFT stages are one launch each, whatever the item order.
#include <limits.h>
#include <math.h>

#include <functional>
#include <new>
#include <vector>

#include "lar_internal.hpp"

using namespace lar;

struct lar_batch {
    std::vector<std::function<hipError_t(hipStream_t)>> steps;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

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

struct Layout {
    size_t table, rowoff, grids, specs, mouts, raster, total;
    std::vector<size_t> grid_at, spec_at, mout_at;   // per item
    std::vector<size_t> type_grid, type_spec, type_mout;
    std::vector<int> type_count;
    int64_t total_sub = 0, total_rows_out = 0;
};

int layout(const lar_plane* planes, int n_types, const lar_batch_item* items, int n_items,
           const lar_fluct* fluct, Layout& L) {
    if (!planes || n_types < 1 || !items || n_items < 1) return LAR_EINVAL;
    if (n_items >= (1 << 27)) return LAR_ESIZE;   // item index shares a 32-bit word with queue marks
    if (fluct && (fluct->mode < 0 || fluct->mode > 3)) return LAR_EINVAL;
    for (int t = 0; t < n_types; ++t) {
        if (!plane_ok(planes[t])) return LAR_ESIZE;
        // a drawn bin's counter word is m * n_ticks + j
        if (fluct && fluct->mode != 0 &&
            (int64_t)planes[t].n_wires * planes[t].n_imp * planes[t].n_ticks > (int64_t)UINT32_MAX)
            return LAR_ESIZE;
    }
    L.type_count.assign(n_types, 0);
    int64_t total_depos = 0;
    for (int i = 0; i < n_items; ++i) {
        const lar_batch_item& it = items[i];
        if (it.plane_type < 0 || it.plane_type >= n_types || it.n_depos < 0 || it.depo_offset < 0 ||
            it.wave_offset < 0 || it.plane >= 256u)
            return LAR_EINVAL;
        if (it.n_depos > (int64_t)UINT32_MAX) return LAR_ESIZE;
        L.type_count[it.plane_type]++;
        L.total_sub += raster_subchunks(it.n_depos);
        L.total_rows_out += planes[it.plane_type].n_wires;
        total_depos += it.n_depos;
    }
    size_t off = 0;
    L.table = off;  off += al(sizeof(RasterItem) * (size_t)n_items);
    L.rowoff = off; off += al(sizeof(int64_t) * (size_t)L.total_rows_out);
    // per type blocks, items of a type in item order
    L.type_grid.assign(n_types, 0);
    L.type_spec.assign(n_types, 0);
    L.type_mout.assign(n_types, 0);
    std::vector<size_t> gsz(n_types), ssz(n_types), msz(n_types);
    for (int t = 0; t < n_types; ++t) {
        const lar_plane& p = planes[t];
        gsz[t] = al((size_t)p.n_wires * p.n_imp * p.n_ticks * sizeof(float));
        ssz[t] = al((size_t)p.n_wires * p.n_imp * spec_ld_of(p) * sizeof(float2));
        msz[t] = al((size_t)p.n_wires * spec_ld_of(p) * sizeof(float2));
    }
    L.grids = off;
    for (int t = 0; t < n_types; ++t) { L.type_grid[t] = off; off += gsz[t] * L.type_count[t]; }
    L.specs = off;
    for (int t = 0; t < n_types; ++t) { L.type_spec[t] = off; off += ssz[t] * L.type_count[t]; }
    L.mouts = off;
    for (int t = 0; t < n_types; ++t) { L.type_mout[t] = off; off += msz[t] * L.type_count[t]; }
    L.grid_at.resize(n_items);
    L.spec_at.resize(n_items);
    L.mout_at.resize(n_items);
    std::vector<int> rank(n_types, 0);
    for (int i = 0; i < n_items; ++i) {
        const int t = items[i].plane_type;
        L.grid_at[i] = L.type_grid[t] + gsz[t] * rank[t];
        L.spec_at[i] = L.type_spec[t] + ssz[t] * rank[t];
        L.mout_at[i] = L.type_mout[t] + msz[t] * rank[t];
        rank[t]++;
    }
    L.raster = off;
    if (fluct && fluct->mode != 0)
        off += raster_ws_fixed_subs(L.total_sub) +
               (fluct->mode == 3 ? 0 : al(((size_t)total_depos * 48 + 4096) * kDeferredBytes));
    L.total = off;
    return LAR_OK;
}

}  // namespace

extern "C" {

int lar_batch_workspace(const lar_plane* planes, int32_t n_types, const lar_batch_item* items,
                        int32_t n_items, const lar_fluct* fluct, size_t* bytes) {
    if (!bytes) return LAR_EINVAL;
    Layout L;
    int st = layout(planes, n_types, items, n_items, fluct, L);
    if (st) return st;
    *bytes = L.total;
    return LAR_OK;
}

int lar_batch_create(const lar_plane* planes, int32_t n_types, const float* const* resp,
                     const lar_depos* depos, float nsigma, const lar_fluct* fluct,
                     const lar_batch_item* items, int32_t n_items, float* wave, void* ws,
                     size_t ws_bytes, int32_t use_graph, lar_batch** out) {
    if (!out || !resp || !depos || !wave || !(nsigma > 0.f) || !isfinite(nsigma)) return LAR_EINVAL;
    *out = nullptr;
    Layout L;
    int st = layout(planes, n_types, items, n_items, fluct, L);
    if (st) return st;
    for (int t = 0; t < n_types; ++t)
        if (L.type_count[t] && !resp[t]) return LAR_EINVAL;
    int64_t total_depos = 0;
    for (int i = 0; i < n_items; ++i)
        total_depos = items[i].depo_offset + items[i].n_depos > total_depos
                          ? items[i].depo_offset + items[i].n_depos
                          : total_depos;
    if (total_depos > depos->n) return LAR_EINVAL;
    if (depos->n > 0 && (!depos->q || !depos->t || !depos->x || !depos->sigma_t || !depos->sigma_x))
        return LAR_EINVAL;
    if (!ws || ws_bytes < L.total || reinterpret_cast<uintptr_t>(ws) % 256) return LAR_EWORKSPACE;
    char* W = reinterpret_cast<char*>(ws);
    const int mode = fluct ? fluct->mode : 0;

    // ---- tables (host), uploaded once
    std::vector<RasterItem> tab(n_items);
    std::vector<int64_t> rowoff;
    rowoff.reserve(L.total_rows_out);
    bool even = true;
    int64_t sub = 0;
    for (int i = 0; i < n_items; ++i) {
        const lar_batch_item& it = items[i];
        const lar_plane& p = planes[it.plane_type];
        RasterItem& r = tab[i];
        r.A.n_ticks = p.n_ticks;
        r.A.n_rows = p.n_wires * p.n_imp;
        r.A.ld = p.n_ticks;
        r.A.org_t = (double)p.t0;
        r.A.wd_t = (double)p.tick;
        r.A.org_x = (double)p.x0 - (double)p.pitch / 2.0;
        r.A.wd_x = (double)p.pitch / (double)p.n_imp;
        r.A.nsig = (double)nsigma;
        r.A.mode = mode;
        r.A.event = it.event;
        r.A.plane = it.plane;
        r.A.seed = fluct ? fluct->seed : 0ull;
        r.q = depos->q + it.depo_offset;
        r.t = depos->t + it.depo_offset;
        r.x = depos->x + it.depo_offset;
        r.st = depos->sigma_t + it.depo_offset;
        r.sx = depos->sigma_x + it.depo_offset;
        r.grid = reinterpret_cast<float*>(W + L.grid_at[i]);
        r.n = it.n_depos;
        r.sub_begin = sub;
        sub += raster_subchunks(it.n_depos);
    }
    // waveform rows of each type, in the order of that type's items
    std::vector<int64_t> type_row0(n_types, 0);
    {
        int64_t acc = 0;
        for (int t = 0; t < n_types; ++t) {
            type_row0[t] = acc;
            acc += (int64_t)L.type_count[t] * planes[t].n_wires;
        }
        rowoff.assign(acc, 0);
        std::vector<int> rank(n_types, 0);
        for (int i = 0; i < n_items; ++i) {
            const int t = items[i].plane_type;
            const lar_plane& p = planes[t];
            for (int w = 0; w < p.n_wires; ++w) {
                int64_t o = items[i].wave_offset + (int64_t)w * p.n_ticks;
                rowoff[type_row0[t] + (int64_t)rank[t] * p.n_wires + w] = o;
                if (o % 2) even = false;
            }
            rank[t]++;
        }
    }
    if (hipMemcpy(W + L.table, tab.data(), sizeof(RasterItem) * n_items, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(W + L.rowoff, rowoff.data(), sizeof(int64_t) * rowoff.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
        return LAR_EHIP;

    lar_batch* b = new (std::nothrow) lar_batch;
    if (!b) return LAR_EINVAL;
    // ---- the launch sequence
    const RasterItem* dtab = reinterpret_cast<const RasterItem*>(W + L.table);
    const int64_t* drow = reinterpret_cast<const int64_t*>(W + L.rowoff);
    float* grids = reinterpret_cast<float*>(W + L.grids);
    const int64_t grid_floats = (int64_t)((L.specs - L.grids) / sizeof(float));
    b->steps.push_back([=](hipStream_t s) { return launch_fill(grids, grid_floats, s); });
    const RasterItem one = tab[0];
    const int64_t total_sub = L.total_sub;
    void* rws = W + L.raster;
    const size_t rws_bytes = L.total - L.raster;
    b->steps.push_back([=](hipStream_t s) {
        return launch_raster_items(mode, one, dtab, n_items, total_sub, rws, rws_bytes, s);
    });
    for (int t = 0; t < n_types; ++t) {
        const int k = L.type_count[t];
        if (!k) continue;
        const lar_plane p = planes[t];
        const int64_t ld = spec_ld_of(p);
        const int rows = p.n_wires * p.n_imp;
        const float* g = reinterpret_cast<const float*>(W + L.type_grid[t]);
        float2* S = reinterpret_cast<float2*>(W + L.type_spec[t]);
        float2* M = reinterpret_cast<float2*>(W + L.type_mout[t]);
        const int64_t gstride = (int64_t)(al((size_t)rows * p.n_ticks * sizeof(float)) / sizeof(float));
        const int64_t sstride = (int64_t)(al((size_t)rows * ld * sizeof(float2)) / sizeof(float2));
        const int64_t mstride = (int64_t)(al((size_t)p.n_wires * ld * sizeof(float2)) / sizeof(float2));
        const float2* R = reinterpret_cast<const float2*>(resp[t]);
        const int F = p.nt_fft / 2 + 1;
        const float scale = (float)(1.0 / ((double)p.nw_fft * (double)p.nt_fft));
        const int64_t* ro = drow + type_row0[t];
        const Sched sc = sched_for(p.n_wires, p.n_imp, p.n_ticks, p.nt_fft, p.nw_fft);
        // grids of one type are gstride apart: contiguous rows when padded to none
        if (gstride == (int64_t)rows * p.n_ticks && sstride == (int64_t)rows * ld) {
            b->steps.push_back([=](hipStream_t s) {
                return launch_r2c_rows(g, p.n_ticks, p.n_ticks, rows * k, p.nt_fft, S, ld, s,
                                       sc.row_threads, sc.row_order);
            });
        } else {
            for (int r = 0; r < k; ++r)
                b->steps.push_back([=](hipStream_t s) {
                    return launch_r2c_rows(g + r * gstride, p.n_ticks, p.n_ticks, rows, p.nt_fft,
                                           S + r * sstride, ld, s, sc.row_threads, sc.row_order);
                });
        }
        b->steps.push_back([=](hipStream_t s) {
            return launch_wire_fused(S, ld, p.n_wires, p.n_imp, p.nw_fft, F, R, M, ld, s, k, sstride,
                                     mstride, sc.wire_cols, sc.wire_threads, sc.wire_order);
        });
        if (mstride == (int64_t)p.n_wires * ld) {
            b->steps.push_back([=](hipStream_t s) {
                return launch_c2r_rows(M, ld, p.n_wires * k, p.nt_fft, wave, p.n_ticks, p.n_ticks, scale,
                                       s, ro, even, sc.row_threads, sc.row_order);
            });
        } else {
            for (int r = 0; r < k; ++r)
                b->steps.push_back([=](hipStream_t s) {
                    return launch_c2r_rows(M + r * mstride, ld, p.n_wires, p.nt_fft, wave, p.n_ticks,
                                           p.n_ticks, scale, s, ro + (int64_t)r * p.n_wires, even,
                                           sc.row_threads, sc.row_order);
                });
        }
    }
    if (use_graph) {
        hipStream_t cs = nullptr;
        bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            for (auto& f : b->steps) ok = ok && f(cs) == hipSuccess;
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
        if (cs) (void)hipStreamDestroy(cs);
        if (!ok) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            delete b;
            return LAR_EHIP;
        }
    }
    *out = b;
    return LAR_OK;
}

int lar_batch_run(lar_batch* b, void* stream) {
    if (!b) return LAR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        hipError_t e = hipGraphLaunch(b->exec, s);
        return e == hipSuccess ? LAR_OK : ((void)hipGetLastError(), LAR_EHIP);
    }
    for (auto& f : b->steps)
        if (f(s) != hipSuccess) return LAR_EHIP;
    return LAR_OK;
}

int lar_batch_destroy(lar_batch* b) {
    if (!b) return LAR_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return LAR_OK;
}

}  // extern "C"
