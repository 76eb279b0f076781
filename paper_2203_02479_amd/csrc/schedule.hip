// schedule.hip -- per-shape launch schedules of the FFT convolution.
//
// A schedule picks, for one plane shape, the workgroup size and radix order
// of the time-axis row transforms, the tile width, workgroup size and
// radix order of the fused wire pass, and the size of the raster's per-wave
// LDS tile.  Every choice gives the same
// transform up to rounding; the fastest one depends on the shape and is
// found by timing (the Python autotuner), then registered here.  Lookups
// happen when a call launches its kernels (a batch plan reads them when it
// is created).
#include <map>
#include <mutex>
#include <tuple>

#include "lar_internal.hpp"

namespace lar {

namespace {
using Key = std::tuple<int, int, int, int, int>;   // n_wires, n_imp, n_ticks, nt_fft, nw_fft
std::mutex g_mu;
std::map<Key, Sched> g_table;

Key key_of(int n_wires, int n_imp, int n_ticks, int nt_fft, int nw_fft) {
    return Key(n_wires, n_imp, n_ticks, nt_fft, nw_fft);
}

Sched sched_default(int nt_fft, int nw_fft) {
    Sched s;
    s.row_threads = default_row_threads(nt_fft);
    s.row_order = 4;   // radix 8 first, 2 x 3 merged into radix 6
    s.wire_cols = default_wire_cols(nw_fft);
    s.wire_threads = default_wire_threads(nw_fft);
    s.wire_order = default_wire_order(nw_fft);
    s.raster_tile = kRasterTileDefault;
    return s;
}

// Radix order o of an n-point plan is a repeat of an earlier order (for
// example every order of a power of 8).
bool order_repeats(int n, int o) {
    FftPlan a, b;
    if (!make_plan(n, &a, o)) return false;
    for (int e = 0; e < o; ++e) {
        if (!make_plan(n, &b, e) || b.npass != a.npass) continue;
        bool same = true;
        for (int i = 0; i < a.npass; ++i) same = same && a.radix[i] == b.radix[i];
        if (same) return true;
    }
    return false;
}

bool sched_ok(const Sched& s, int nt_fft, int nw_fft) {
    return row_sched_ok(nt_fft, s.row_threads, s.row_order) &&
           wire_sched_ok(nw_fft, s.wire_cols, s.wire_threads, s.wire_order) && raster_tile_ok(s.raster_tile);
}
}  // namespace

Sched sched_for(int n_wires, int n_imp, int n_ticks, int nt_fft, int nw_fft) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(key_of(n_wires, n_imp, n_ticks, nt_fft, nw_fft));
        if (it != g_table.end()) return it->second;
    }
    return sched_default(nt_fft, nw_fft);
}

}  // namespace lar

using namespace lar;

static int check_shape(const lar_plane* p) {
    if (!p || p->n_wires < 1 || p->n_imp < 1 || p->n_ticks < 1) return LAR_EINVAL;
    if (p->nt_fft < 2 || p->nt_fft % 2 || p->nt_fft > 16384 || p->nt_fft < p->n_ticks) return LAR_ESIZE;
    if (p->nw_fft < p->n_wires || p->nw_fft > 1024) return LAR_ESIZE;
    FftPlan a, b;
    if (!make_plan(p->nt_fft / 2, &a) || !make_plan(p->nw_fft, &b)) return LAR_ESIZE;
    return LAR_OK;
}

static Sched from_abi(const lar_schedule* s) {
    Sched r;
    r.row_threads = s->row_threads;
    r.row_order = s->row_order;
    r.wire_cols = s->wire_cols;
    r.wire_threads = s->wire_threads;
    r.wire_order = s->wire_order;
    r.raster_tile = s->raster_tile ? s->raster_tile : kRasterTileDefault;
    return r;
}

static void to_abi(const Sched& s, lar_schedule* r) {
    r->row_threads = s.row_threads;
    r->row_order = s.row_order;
    r->wire_cols = s.wire_cols;
    r->wire_threads = s.wire_threads;
    r->wire_order = s.wire_order;
    r->raster_tile = s.raster_tile;
}

extern "C" {

int lar_schedule_default(const lar_plane* p, lar_schedule* out) {
    int st;
    if ((st = check_shape(p))) return st;
    if (!out) return LAR_EINVAL;
    to_abi(sched_default(p->nt_fft, p->nw_fft), out);
    return LAR_OK;
}

int lar_schedule_get(const lar_plane* p, lar_schedule* out) {
    int st;
    if ((st = check_shape(p))) return st;
    if (!out) return LAR_EINVAL;
    to_abi(sched_for(p->n_wires, p->n_imp, p->n_ticks, p->nt_fft, p->nw_fft), out);
    return LAR_OK;
}

int lar_schedule_set(const lar_plane* p, const lar_schedule* s) {
    int st;
    if ((st = check_shape(p))) return st;
    const Key k = key_of(p->n_wires, p->n_imp, p->n_ticks, p->nt_fft, p->nw_fft);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!s) {
        g_table.erase(k);
        return LAR_OK;
    }
    const Sched v = from_abi(s);
    if (!sched_ok(v, p->nt_fft, p->nw_fft)) return LAR_EINVAL;
    g_table[k] = v;
    return LAR_OK;
}

int lar_schedule_candidates(const lar_plane* p, lar_schedule* out, int32_t cap, int32_t* n) {
    int st;
    if ((st = check_shape(p))) return st;
    if (!n || cap < 0 || (cap > 0 && !out)) return LAR_EINVAL;
    static const int row_threads[5] = {256, 384, 512, 768, 1024};
    static const int threads[4] = {256, 512, 576, 1024};   // 576: 4 columns, Wf 864's 6 4 6 6 plan
    static const int cols[3] = {4, 8, 16};
    const Sched d = sched_default(p->nt_fft, p->nw_fft);
    int count = 0;
    auto same = [](const Sched& a, const Sched& b) {
        return a.row_threads == b.row_threads && a.row_order == b.row_order &&
               a.wire_cols == b.wire_cols && a.wire_threads == b.wire_threads &&
               a.wire_order == b.wire_order && a.raster_tile == b.raster_tile;
    };
    auto emit = [&](const Sched& s) {
        if (!sched_ok(s, p->nt_fft, p->nw_fft)) return;
        if (count < cap) to_abi(s, out + count);
        ++count;
    };
    emit(d);   // the built-in schedule first

    // row choices with the default wire pass, then wire choices with the
    // default rows: the two stages are timed apart, so the candidate list is
    // their union rather than their product
    for (int t : row_threads)
        for (int o = 0; o < kPlanOrders; ++o) {
            if (order_repeats(p->nt_fft / 2, o)) continue;
            Sched s = d;
            s.row_threads = t;
            s.row_order = o;
            if (!same(s, d)) emit(s);
        }
    for (int c : cols)
        for (int t : threads)
            for (int o = 0; o < kPlanOrders; ++o) {
                if (order_repeats(p->nw_fft, o)) continue;
                Sched s = d;
                s.wire_cols = c;
                s.wire_threads = t;
                s.wire_order = o;
                if (!same(s, d)) emit(s);
            }
    // raster tiles with the default FFT choices
    for (int t : {384, 640, 768}) {
        Sched s = d;
        s.raster_tile = t;
        if (!same(s, d)) emit(s);
    }
    *n = count;
    return LAR_OK;
}

}  // extern "C"
