// Host core of the gate-level re-simulator: validation, delay-arc
// compilation, levelization orchestration, window planning and the level
// schedule, behind the C ABI declared in include/gatesim.h.
#include "gatesim.h"
#include "internal.h"
#include "host.h"

#include <algorithm>
#include <map>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace gs;

static thread_local std::string g_tls_err;

gs_status gs_fail(gs_ctx *ctx, gs_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_tls_err = buf;
    return code;
}

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return gs_fail(ctx, GS_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

uint64_t gs_now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---------------------------------------------------------------------------
// host-only validation
// ---------------------------------------------------------------------------
static gs_status check_netlist_impl(gs_ctx *ctx, int32_t n_cells, const uint8_t *n_pins, int32_t n_inputs,
                                    int32_t n_gates, const int32_t *cell_of_gate, const int64_t *fanin_ptr,
                                    const int32_t *fanin_net)
{
    if (n_inputs < 0 || n_gates < 0) return gs_fail(ctx, GS_E_INVALID, "negative netlist size");
    if ((int64_t)n_inputs + n_gates > (int64_t)0x1fffffff) return gs_fail(ctx, GS_E_INVALID, "too many nets");
    if (n_gates > 0 && (!cell_of_gate || !fanin_ptr || !fanin_net))
        return gs_fail(ctx, GS_E_INVALID, "null netlist array");
    if (n_gates > 0 && fanin_ptr[0] != 0) return gs_fail(ctx, GS_E_INVALID, "fanin_ptr[0] must be 0");
    const int64_t N = (int64_t)n_inputs + n_gates;
    for (int32_t g = 0; g < n_gates; g++) {
        int32_t c = cell_of_gate[g];
        if (c < 0 || c >= n_cells) return gs_fail(ctx, GS_E_INVALID, "gate %d: cell %d out of range", g, c);
        int64_t k = fanin_ptr[g + 1] - fanin_ptr[g];
        if (k != n_pins[c])
            return gs_fail(ctx, GS_E_INVALID, "gate %d: %lld fanins but cell %d has %d pins", g, (long long)k, c,
                           (int)n_pins[c]);
        for (int64_t s = fanin_ptr[g]; s < fanin_ptr[g + 1]; s++)
            if (fanin_net[s] < 0 || fanin_net[s] >= N)
                return gs_fail(ctx, GS_E_INVALID, "gate %d pin %lld: net %d out of range", g,
                               (long long)(s - fanin_ptr[g]), fanin_net[s]);
    }
    return GS_OK;
}

static gs_status check_cells(gs_ctx *ctx, int32_t n_cells, const uint8_t *n_pins)
{
    if (n_cells <= 0 || !n_pins) return gs_fail(ctx, GS_E_INVALID, "no cells");
    for (int32_t c = 0; c < n_cells; c++)
        if (n_pins[c] < 1 || n_pins[c] > 6) return gs_fail(ctx, GS_E_INVALID, "cell %d: pin count %d not in 1..6", c, n_pins[c]);
    return GS_OK;
}

extern "C" gs_status gs_check_netlist(int32_t n_cells, const uint8_t *n_pins, int32_t n_inputs, int32_t n_gates,
                                      const int32_t *cell_of_gate, const int64_t *fanin_ptr, const int32_t *fanin_net)
{
    gs_status st = check_cells(nullptr, n_cells, n_pins);
    if (st) return st;
    return check_netlist_impl(nullptr, n_cells, n_pins, n_inputs, n_gates, cell_of_gate, fanin_ptr, fanin_net);
}

// Compiles arc records into one delay row per fanin slot (q, and 8 delays
// in PinRec::d order): in each (condition value, input edge) combination
// the most specific record applies, as arc_winner picks it.
static gs_status compile_arcs(gs_ctx *ctx, const std::vector<uint8_t> &gate_k, const std::vector<int64_t> &fanin_ptr,
                              int64_t n_arcs, const gs_arc *arcs, std::vector<int32_t> &q, std::vector<int32_t> &dl,
                              int32_t *max_delay, int32_t *zero_delay, std::vector<int64_t> *rec_out = nullptr)
{
    const int32_t G = (int32_t)gate_k.size();
    const int64_t F = G ? fanin_ptr[G] : 0;
    if (n_arcs < 0 || (n_arcs > 0 && !arcs)) return gs_fail(ctx, GS_E_INVALID, "bad arc array");
    std::vector<int64_t> local;
    std::vector<int64_t> &rec = rec_out ? *rec_out : local;
    rec.assign(kArcKinds * (size_t)F, -1);
    q.assign(F, -1);
    int64_t n_zero = 0, n_pos = 0;
    int32_t mx = 0;
    for (int64_t a = 0; a < n_arcs; a++) {
        const gs_arc &r = arcs[a];
        if (r.gate < 0 || r.gate >= G) return gs_fail(ctx, GS_E_INVALID, "arc %lld: gate %d out of range", (long long)a, r.gate);
        const int k = gate_k[r.gate];
        if (r.pin < 0 || r.pin >= k) return gs_fail(ctx, GS_E_INVALID, "arc %lld: pin %d out of range", (long long)a, r.pin);
        if (r.rise_ps < 0 || r.fall_ps < 0) return gs_fail(ctx, GS_E_INVALID, "arc %lld: negative delay", (long long)a);
        if (r.rise_ps > (1 << 24) || r.fall_ps > (1 << 24))
            return gs_fail(ctx, GS_E_INVALID, "arc %lld: delay above 2^24 ps", (long long)a);
        n_zero += (r.rise_ps == 0) + (r.fall_ps == 0);
        n_pos += (r.rise_ps > 0) + (r.fall_ps > 0);
        mx = std::max(mx, std::max(r.rise_ps, r.fall_ps));
        const int64_t s = fanin_ptr[r.gate] + r.pin;
        if (r.in_edge < 0 || r.in_edge > 2)
            return gs_fail(ctx, GS_E_INVALID, "arc %lld: input-edge qualifier must be 0, 1 or 2", (long long)a);
        if (r.cond_pin >= 0) {
            if (r.cond_pin >= k || r.cond_pin == r.pin)
                return gs_fail(ctx, GS_E_INVALID, "arc %lld: bad condition pin %d", (long long)a, r.cond_pin);
            if (r.cond_val != 0 && r.cond_val != 1)
                return gs_fail(ctx, GS_E_INVALID, "arc %lld: condition value must be 0 or 1", (long long)a);
            if (q[s] >= 0 && q[s] != r.cond_pin)
                return gs_fail(ctx, GS_E_INVALID, "gate %d pin %d: conditional arcs on more than one condition pin",
                               r.gate, r.pin);
            q[s] = r.cond_pin;
        }
        int64_t &slot = rec[kArcKinds * s + arc_kind(r)];
        slot = slot == -1 ? a : -2;
    }
    if (n_zero > 0 && n_pos > 0)
        return gs_fail(ctx, GS_E_INVALID, "gate delays must be all >= 1, or all 0 (zero-delay mode)");
    dl.assign(8 * (size_t)F, 0);
    for (int32_t g = 0; g < G; g++)
        for (int64_t s = fanin_ptr[g]; s < fanin_ptr[g + 1]; s++) {
            for (int cv = 0; cv < 2; cv++)
                for (int ie = 0; ie < 2; ie++) {
                    const int64_t w = arc_winner(&rec[kArcKinds * s], cv, ie);
                    if (w == -1)
                        return gs_fail(ctx, GS_E_INVALID, "gate %d pin %lld: a pin state has no arc record", g,
                                       (long long)(s - fanin_ptr[g]));
                    if (w == -2)
                        return gs_fail(ctx, GS_E_INVALID, "gate %d pin %lld: two arc records apply to one pin state",
                                       g, (long long)(s - fanin_ptr[g]));
                    dl[8 * s + gs::delay_slot(cv, ie, 1)] = arcs[w].rise_ps;
                    dl[8 * s + gs::delay_slot(cv, ie, 0)] = arcs[w].fall_ps;
                }
            if (q[s] < 0) q[s] = 0;
        }
    *max_delay = mx;
    *zero_delay = (n_pos == 0) ? 1 : 0;
    return GS_OK;
}

extern "C" gs_status gs_check_arcs(int32_t n_cells, const uint8_t *n_pins, int32_t n_gates, const int32_t *cell_of_gate,
                                   int64_t n_arcs, const gs_arc *arcs)
{
    gs_status st = check_cells(nullptr, n_cells, n_pins);
    if (st) return st;
    std::vector<uint8_t> k(n_gates);
    std::vector<int64_t> fp(n_gates + 1, 0);
    for (int32_t g = 0; g < n_gates; g++) {
        if (cell_of_gate[g] < 0 || cell_of_gate[g] >= n_cells) return gs_fail(nullptr, GS_E_INVALID, "cell out of range");
        k[g] = n_pins[cell_of_gate[g]];
        fp[g + 1] = fp[g] + k[g];
    }
    std::vector<int32_t> q, dl;
    int32_t mx, zd;
    return compile_arcs(nullptr, k, fp, n_arcs, arcs, q, dl, &mx, &zd);
}

static gs_status check_stim_impl(gs_ctx *ctx, int32_t n_inputs, int32_t period, int32_t n_cycles, const uint8_t *init,
                                 const int64_t *tp, const int64_t *ts)
{
    if (period < 1 || period > (1 << 24)) return gs_fail(ctx, GS_E_INVALID, "period must be in 1..2^24 ps");
    if (n_cycles < 0) return gs_fail(ctx, GS_E_INVALID, "negative cycle count");
    if (n_inputs > 0 && (!init || !tp)) return gs_fail(ctx, GS_E_INVALID, "null stimulus array");
    if (n_inputs > 0 && tp[0] != 0) return gs_fail(ctx, GS_E_INVALID, "toggle_ptr[0] must be 0");
    const int64_t end = (int64_t)n_cycles * period;
    for (int32_t i = 0; i < n_inputs; i++) {
        if (init[i] > 1) return gs_fail(ctx, GS_E_INVALID, "input %d: initial value must be 0 or 1", i);
        if (tp[i + 1] < tp[i]) return gs_fail(ctx, GS_E_INVALID, "toggle_ptr not non-decreasing at input %d", i);
        for (int64_t k = tp[i]; k < tp[i + 1]; k++) {
            if (ts[k] < 0 || ts[k] >= end)
                return gs_fail(ctx, GS_E_INVALID, "input %d: toggle at %lld outside [0, %lld)", i, (long long)ts[k],
                               (long long)end);
            if (k > tp[i] && ts[k] <= ts[k - 1])
                return gs_fail(ctx, GS_E_INVALID, "input %d: toggle times not strictly increasing", i);
        }
    }
    return GS_OK;
}

extern "C" gs_status gs_check_stimulus(int32_t n_inputs, int32_t period_ps, int32_t n_cycles, const uint8_t *init,
                                       const int64_t *toggle_ptr, const int64_t *toggle_ps)
{
    return check_stim_impl(nullptr, n_inputs, period_ps, n_cycles, init, toggle_ptr, toggle_ps);
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" void gs_default_options(gs_options *o)
{
    std::memset(o, 0, sizeof(*o));
    o->lds_cap = 0;
    o->waves_per_block = 4;
    o->tiles_per_wave = 8;
    o->schedule = GS_SCHED_LEVELS;
}

static gs_status dev_alloc(gs_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) return GS_OK;
    if (ctx && ctx->noalloc)
        return gs_fail(ctx, GS_E_NOMEM, "the allocation-free call needs %zu more bytes than its static scratch "
                       "holds", bytes);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return gs_fail(ctx, GS_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    return GS_OK;
}

void gs_dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

extern "C" gs_status gs_create(const gs_options *opt, gs_ctx **out)
{
    if (!out) return gs_fail(nullptr, GS_E_INVALID, "null output pointer");
    *out = nullptr;
    gs_options o;
    if (opt) o = *opt;
    else gs_default_options(&o);
    const bool auto_cap = o.lds_cap == 0;
    if (o.lds_cap == 0) o.lds_cap = 8;
    if (o.waves_per_block == 0) o.waves_per_block = 4;
    if (o.tiles_per_wave == 0) o.tiles_per_wave = 8;
    if (o.tiles_per_wave < 1 || o.tiles_per_wave > 64) return gs_fail(nullptr, GS_E_INVALID, "tiles_per_wave must be 1..64");
    if (o.lds_cap != 4 && o.lds_cap != 8 && o.lds_cap != 16 && o.lds_cap != 24 && o.lds_cap != 32)
        return gs_fail(nullptr, GS_E_INVALID, "lds_cap must be 4, 8, 16, 24 or 32");
    if (o.waves_per_block < 1 || o.waves_per_block > 8) return gs_fail(nullptr, GS_E_INVALID, "waves_per_block must be 1..8");
    if (o.schedule != GS_SCHED_LEVELS && o.schedule != GS_SCHED_GRAPH) return gs_fail(nullptr, GS_E_INVALID, "bad schedule");
    if (o.window_cycles < 0) return gs_fail(nullptr, GS_E_INVALID, "negative window");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return gs_fail(nullptr, GS_E_DEVICE, "no HIP device available");
    }
    if (o.device < 0 || o.device >= ndev) return gs_fail(nullptr, GS_E_DEVICE, "device %d not present", o.device);
    if (hipSetDevice(o.device) != hipSuccess) return gs_fail(nullptr, GS_E_DEVICE, "hipSetDevice failed");
    int lim = 0;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, o.device) != hipSuccess || lim <= 0) {
        (void)hipGetLastError();
        lim = 65536;
    }
    if (!auto_cap && gate_eval_lds_bytes(o.lds_cap, o.waves_per_block) > (size_t)lim)
        return gs_fail(nullptr, GS_E_INVALID, "lds_cap %d with %d waves per block needs %zu bytes of LDS per block; "
                       "the device allows %d", o.lds_cap, o.waves_per_block,
                       gate_eval_lds_bytes(o.lds_cap, o.waves_per_block), lim);
    gs_ctx *ctx = new gs_ctx();
    ctx->opt = o;
    ctx->auto_cap = auto_cap;
    ctx->lds_limit = (size_t)lim;
    if (o.stream) {
        ctx->stream = (hipStream_t)o.stream;
        ctx->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return gs_fail(nullptr, GS_E_DEVICE, "hipStreamCreate failed");
        }
        ctx->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return gs_fail(nullptr, GS_E_DEVICE, "hipStreamCreate failed");
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        fr = 0;
    }
    ctx->budget = o.hbm_budget ? o.hbm_budget : (uint64_t)(0.8 * (double)fr);
    if (o.arena) ctx->budget = o.arena_bytes;
    void *p;
    if (dev_alloc(ctx, &p, 64) != GS_OK) {
        gs_destroy(ctx);
        return gs_fail(nullptr, GS_E_NOMEM, "small allocation failed");
    }
    ctx->d_misc = (unsigned long long *)p;   // [1..2] flags, [4..] counters
    if (dev_alloc(ctx, &p, sizeof(unsigned long long) * kMaxStripes * kBumpStride) != GS_OK) {
        gs_destroy(ctx);
        return gs_fail(nullptr, GS_E_NOMEM, "small allocation failed");
    }
    ctx->d_bump = (unsigned long long *)p;
    // this device's static scratch (allocation-free simulate), looked up now
    // while the device is current
    hipError_t se = scratch_region(o.device, &p);
    if (se != hipSuccess) {
        (void)hipGetLastError();
        gs_destroy(ctx);
        return gs_fail(nullptr, GS_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(se));
    }
    ctx->d_scratch = (char *)p;
    *out = ctx;
    return GS_OK;
}

extern "C" gs_status gs_destroy(gs_ctx *ctx)
{
    if (!ctx) return GS_OK;
    gs_serve_shutdown(ctx);
    (void)hipSetDevice(ctx->opt.device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (Design *d : ctx->designs) {
        if (!d) continue;
        gs_dev_free(d->d_fanin_ptr); gs_dev_free(d->d_fanin_net); gs_dev_free(d->d_level);
        gs_dev_free(d->d_gates); gs_dev_free(d->d_pins); gs_dev_free(d->d_saif); gs_dev_free(d->d_stage);
        delete d;
    }
    for (Stim *s : ctx->stims) {
        if (!s) continue;
        if (s->owns) { gs_dev_free(s->d_init); gs_dev_free(s->d_tp); gs_dev_free(s->d_ts); }
        delete s;
    }
    gs_window_release(ctx, &ctx->win);
    gs_dev_free(ctx->d_segs);
    gs_dev_free(ctx->d_misc);
    gs_dev_free(ctx->d_bump);
    gs_dev_free(ctx->d_regions);
    gs_dev_free(ctx->d_rbump);
    for (auto &ev : ctx->events) (void)hipEventDestroy(ev);
    gs_graph_cache_clear(ctx);
    gs_dev_free(ctx->d_c0);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GS_OK;
}

extern "C" const char *gs_last_error(gs_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_tls_err.c_str();
}

extern "C" gs_status gs_load_cells(gs_ctx *ctx, int32_t n_cells, const uint8_t *n_pins, const uint64_t *truth)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    gs_status st = check_cells(ctx, n_cells, n_pins);
    if (st) return st;
    if (!truth) return gs_fail(ctx, GS_E_INVALID, "null truth table");
    ctx->cell_k.assign(n_pins, n_pins + n_cells);
    ctx->cell_truth.assign(truth, truth + n_cells);
    for (int32_t c = 0; c < n_cells; c++)
        if (n_pins[c] < 6) ctx->cell_truth[c] &= (1ull << (1u << n_pins[c])) - 1ull;
    return GS_OK;
}

Design *gs_get_design(gs_ctx *ctx, int32_t id)
{
    if (id < 0 || id >= (int32_t)ctx->designs.size()) return nullptr;
    return ctx->designs[id];
}

// Levelizes on the GPU and buckets gates by level (perm = level order).
static gs_status levelize(gs_ctx *ctx, Design *d)
{
    hipStream_t s = ctx->stream;
    const int32_t I = d->I, G = d->G;
    void *p;
    gs_status st;
    if ((st = dev_alloc(ctx, &p, sizeof(int64_t) * (G + 1)))) return st;
    d->d_fanin_ptr = (int64_t *)p;
    if ((st = dev_alloc(ctx, &p, sizeof(int32_t) * std::max<int64_t>(1, d->F)))) return st;
    d->d_fanin_net = (int32_t *)p;
    if ((st = dev_alloc(ctx, &p, sizeof(int32_t) * std::max<int64_t>(1, (int64_t)I + G)))) return st;
    d->d_level = (int32_t *)p;
    HIPCHK(hipMemcpyAsync(d->d_fanin_ptr, d->fanin_ptr.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    if (d->F) HIPCHK(hipMemcpyAsync(d->d_fanin_net, d->fanin_net.data(), sizeof(int32_t) * d->F, hipMemcpyHostToDevice, s));
    HIPCHK(launch_level_init(d->d_level, I, G, s));
    int iters = 0;
    if (G) {
        // temporary buffers of the frontier levelizer, freed on return
        struct Temp {
            std::vector<void *> v;
            ~Temp() { for (void *q : v) gs_dev_free(q); }
        } tmp;
        auto take = [&](size_t bytes, void **q) {
            gs_status r = dev_alloc(ctx, q, std::max<size_t>(bytes, 8));
            if (!r) tmp.v.push_back(*q);
            return r;
        };
        void *pp[7];
        if ((st = take(sizeof(unsigned int) * G, &pp[0])) || (st = take(sizeof(unsigned int) * G, &pp[1])) ||
            (st = take(sizeof(int64_t) * ((size_t)G + 1), &pp[2])) || (st = take(sizeof(int32_t) * (size_t)d->F, &pp[3])) ||
            (st = take(sizeof(int32_t) * G, &pp[4])) || (st = take(sizeof(int32_t) * G, &pp[5])) ||
            (st = take(sizeof(unsigned int) * 2, &pp[6])))
            return st;
        unsigned int *pending = (unsigned int *)pp[0], *fo_cnt = (unsigned int *)pp[1], *sizes = (unsigned int *)pp[6];
        int64_t *fo_ptr = (int64_t *)pp[2];
        int32_t *fo = (int32_t *)pp[3], *cur = (int32_t *)pp[4], *nxt = (int32_t *)pp[5];
        // sink lists of the gate outputs: counts, their prefix sum on the host, fill
        HIPCHK(launch_fill_u32(fo_cnt, (uint64_t)G, 0u, s));
        HIPCHK(launch_fanout_count(d->d_fanin_ptr, d->d_fanin_net, I, G, pending, fo_cnt, s));
        std::vector<unsigned int> hc(G);
        HIPCHK(hipMemcpyAsync(hc.data(), fo_cnt, sizeof(unsigned int) * G, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int64_t> hp((size_t)G + 1, 0);
        for (int32_t g = 0; g < G; g++) hp[g + 1] = hp[g] + hc[g];
        HIPCHK(hipMemcpyAsync(fo_ptr, hp.data(), sizeof(int64_t) * ((size_t)G + 1), hipMemcpyHostToDevice, s));
        HIPCHK(launch_fill_u32(fo_cnt, (uint64_t)G, 0u, s));
        HIPCHK(launch_fanout_fill(d->d_fanin_ptr, d->d_fanin_net, I, G, fo_ptr, fo_cnt, fo, s));
        // frontiers, one level each
        unsigned int n = 0;
        HIPCHK(launch_fill_u32(sizes, 2, 0u, s));
        HIPCHK(launch_level_seed(pending, d->d_level, I, G, cur, sizes, s));
        HIPCHK(hipMemcpyAsync(&n, sizes, sizeof(n), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int64_t placed = n;
        while (n > 0) {
            iters++;
            HIPCHK(launch_fill_u32(sizes + 1, 1, 0u, s));
            HIPCHK(launch_level_frontier(cur, n, fo_ptr, fo, d->d_fanin_ptr, d->d_fanin_net, pending, d->d_level, I,
                                         nxt, sizes + 1, s));
            HIPCHK(hipMemcpyAsync(&n, sizes + 1, sizeof(n), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            placed += n;
            std::swap(cur, nxt);
        }
        if (placed < G)
            return gs_fail(ctx, GS_E_NOT_DAG, "netlist has a combinational cycle (%lld gates unplaced)",
                           (long long)(G - placed));
    }
    d->level.resize(G);
    if (G) HIPCHK(hipMemcpyAsync(d->level.data(), d->d_level + I, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t L = 0;
    for (int32_t g = 0; g < G; g++) L = std::max(L, d->level[g]);
    d->L = L;
    // bucket by level on the device: histogram, host prefix sum, scatter
    void *pc;
    if ((st = dev_alloc(ctx, &pc, sizeof(unsigned int) * (L + 2)))) return st;
    unsigned int *cursor = (unsigned int *)pc;
    std::vector<unsigned int> hist(L + 2, 0);
    st = GS_OK;
    do {
        if (hipMemsetAsync(cursor, 0, sizeof(unsigned int) * (L + 2), s) != hipSuccess) { st = GS_E_DEVICE; break; }
        if (launch_level_bucket(d->d_level, I, G, cursor, nullptr, 1, s) != hipSuccess) { st = GS_E_DEVICE; break; }
        if (hipMemcpyAsync(hist.data(), cursor, sizeof(unsigned int) * (L + 2), hipMemcpyDeviceToHost, s) != hipSuccess) { st = GS_E_DEVICE; break; }
        if (hipStreamSynchronize(s) != hipSuccess) { st = GS_E_DEVICE; break; }
        d->level_ptr.assign(L + 2, 0);
        for (int32_t l = 1; l <= L; l++) d->level_ptr[l + 1] = d->level_ptr[l] + hist[l];
        std::vector<unsigned int> start(L + 2, 0);
        for (int32_t l = 0; l <= L; l++) start[l] = d->level_ptr[l];
        d->perm.resize(G);
        void *pp;
        if (dev_alloc(ctx, &pp, sizeof(int32_t) * std::max(1, G)) != GS_OK) { st = GS_E_NOMEM; break; }
        if (hipMemcpyAsync(cursor, start.data(), sizeof(unsigned int) * (L + 2), hipMemcpyHostToDevice, s) != hipSuccess ||
            launch_level_bucket(d->d_level, I, G, cursor, (int32_t *)pp, 0, s) != hipSuccess ||
            (G && hipMemcpyAsync(d->perm.data(), pp, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s) != hipSuccess) ||
            hipStreamSynchronize(s) != hipSuccess)
            st = GS_E_DEVICE;
        gs_dev_free(pp);
    } while (0);
    gs_dev_free(cursor);
    if (st) return gs_fail(ctx, st, "level bucketing failed");
    d->level_sweeps = iters;
    d->level_kmax.assign(L + 2, 0);
    for (int32_t l = 1; l <= L; l++)
        for (uint32_t p = d->level_ptr[l]; p < d->level_ptr[l + 1]; p++)
            d->level_kmax[l] = std::max<int32_t>(d->level_kmax[l], d->gate_k[d->perm[p]]);
    return GS_OK;
}

extern "C" gs_status gs_load_netlist(gs_ctx *ctx, int32_t n_inputs, int32_t n_gates, const int32_t *cell_of_gate,
                                     const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t *design_id)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->cell_k.empty()) return gs_fail(ctx, GS_E_STATE, "load the cell library first");
    gs_status st = check_netlist_impl(ctx, (int32_t)ctx->cell_k.size(), ctx->cell_k.data(), n_inputs, n_gates,
                                      cell_of_gate, fanin_ptr, fanin_net);
    if (st) return st;
    (void)hipSetDevice(ctx->opt.device);
    Design *d = new Design();
    d->I = n_inputs;
    d->G = n_gates;
    d->N = n_inputs + n_gates;
    d->F = n_gates ? fanin_ptr[n_gates] : 0;
    d->gate_k.resize(n_gates);
    d->gate_truth.resize(n_gates);
    for (int32_t g = 0; g < n_gates; g++) {
        d->gate_k[g] = ctx->cell_k[cell_of_gate[g]];
        d->gate_truth[g] = ctx->cell_truth[cell_of_gate[g]];
        d->max_pins = std::max<int32_t>(d->max_pins, d->gate_k[g]);
    }
    d->fanin_ptr.assign(fanin_ptr, fanin_ptr + n_gates + 1);
    if (n_gates == 0) d->fanin_ptr.assign(1, 0);
    d->fanin_net.assign(fanin_net, fanin_net + d->F);
    d->wr.assign(d->F, 0);
    d->wf.assign(d->F, 0);
    void *p;
    if ((st = dev_alloc(ctx, &p, sizeof(unsigned long long) * kSaifArrays * std::max(1, d->N)))) { delete d; return st; }
    d->d_saif = (unsigned long long *)p;
    if ((st = dev_alloc(ctx, &p, sizeof(unsigned long long) * kSaifArrays * std::max(1, d->N)))) { gs_dev_free(d->d_saif); delete d; return st; }
    d->d_stage = (unsigned long long *)p;
    hipError_t e = hipMemsetAsync(d->d_saif, 0, sizeof(unsigned long long) * kSaifArrays * std::max(1, d->N), ctx->stream);
    if (e != hipSuccess) { gs_dev_free(d->d_saif); gs_dev_free(d->d_stage); delete d; return gs_fail(ctx, GS_E_DEVICE, "memset failed"); }
    ctx->designs.push_back(d);
    st = levelize(ctx, d);
    if (st) {
        ctx->designs.back() = nullptr;
        gs_dev_free(d->d_fanin_ptr); gs_dev_free(d->d_fanin_net); gs_dev_free(d->d_level);
        gs_dev_free(d->d_saif); gs_dev_free(d->d_stage);
        delete d;
        return st;
    }
    if (design_id) *design_id = (int32_t)ctx->designs.size() - 1;
    return GS_OK;
}

// Packs the level-ordered gate and pin records and uploads them.
static gs_status pack_design(gs_ctx *ctx, Design *d)
{
    const int32_t G = d->G;
    std::vector<GateRec> gates(std::max(1, G));
    std::vector<PinRec> pins(std::max<int64_t>(1, d->F));
    // the last level that reads each gate output (its own level if none)
    std::vector<int32_t> dead(G);
    for (int32_t g = 0; g < G; g++) dead[g] = d->level[g];
    for (int32_t g = 0; g < G; g++)
        for (int64_t s = d->fanin_ptr[g]; s < d->fanin_ptr[g + 1]; s++) {
            const int32_t n = d->fanin_net[s];
            if (n >= d->I) dead[n - d->I] = std::max(dead[n - d->I], d->level[g]);
        }
    // Arena regions for the release of dead nets: region 0 holds the inputs;
    // a gate output goes to the region of its level and of its last reading
    // level rounded down to a multiple of q (at most 16 such classes per
    // level), so that a region's nets are written by one launch and its space
    // can be reused once the last of them has been read.
    const int32_t q = std::max(1, (d->L + 15) / 16);
    std::map<std::pair<int32_t, int32_t>, int32_t> region_of;
    std::vector<int32_t> gate_region(G);
    d->region_nets.assign(1, d->I);
    d->region_first.assign(1, 0);
    d->region_last.assign(1, INT32_MAX);
    for (int32_t g = 0; g < G; g++) {
        const auto key = std::make_pair(d->level[g], dead[g] / q);
        auto it = region_of.find(key);
        if (it == region_of.end()) {
            it = region_of.emplace(key, (int32_t)d->region_nets.size()).first;
            d->region_nets.push_back(0);
            d->region_first.push_back(d->level[g]);
            d->region_last.push_back(0);
        }
        const int32_t k = it->second;
        gate_region[g] = k;
        d->region_nets[k]++;
        d->region_last[k] = std::max(d->region_last[k], dead[g]);
    }
    d->region_wpp.assign(d->region_nets.size(), 0.0);
    d->region_grow.assign(d->region_nets.size(), 1.0);
    uint32_t pc = 0;
    for (int32_t p = 0; p < G; p++) {
        const int32_t g = d->perm[p];
        GateRec &r = gates[p];
        std::memset(&r, 0, sizeof(r));
        r.out = (uint32_t)(d->I + g);
        r.dead = (uint32_t)gate_region[g];
        r.pin0 = pc;
        r.k = d->gate_k[g];
        r.truth = d->gate_truth[g];
        for (int64_t s = d->fanin_ptr[g]; s < d->fanin_ptr[g + 1]; s++) {
            PinRec &q = pins[pc++];
            q.net = d->fanin_net[s];
            q.q = d->q[s];
            for (int i = 0; i < 8; i++) q.d[i] = d->dl[8 * s + i];
            q.wr = d->wr[s]; q.wf = d->wf[s];
        }
    }
    if (!d->d_gates) {
        void *p;
        gs_status st;
        if ((st = dev_alloc(ctx, &p, sizeof(GateRec) * gates.size()))) return st;
        d->d_gates = (GateRec *)p;
        if ((st = dev_alloc(ctx, &p, sizeof(PinRec) * pins.size()))) return st;
        d->d_pins = (PinRec *)p;
    }
    HIPCHK(hipMemcpyAsync(d->d_gates, gates.data(), sizeof(GateRec) * gates.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d->d_pins, pins.data(), sizeof(PinRec) * pins.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    d->version++;
    return GS_OK;
}

extern "C" gs_status gs_load_arcs(gs_ctx *ctx, int32_t design, int64_t n_arcs, const gs_arc *arcs)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    std::vector<int32_t> q, dl;
    std::vector<int64_t> rec;
    int32_t mx, zd;
    gs_status st = compile_arcs(ctx, d->gate_k, d->fanin_ptr, n_arcs, arcs, q, dl, &mx, &zd, &rec);
    if (st) return st;
    if (zd && d->has_wires) return gs_fail(ctx, GS_E_INVALID, "zero-delay arcs need zero wire delays");
    d->q.swap(q); d->dl.swap(dl);
    d->slot_rec.swap(rec);
    d->arcs.assign(arcs, arcs + n_arcs);
    d->max_delay = mx;
    d->zero_delay = zd;
    d->arcs_loaded = true;
    (void)hipSetDevice(ctx->opt.device);
    return pack_design(ctx, d);
}

extern "C" gs_status gs_load_wires(gs_ctx *ctx, int32_t design, const int32_t *rise_ps, const int32_t *fall_ps)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    if ((rise_ps == nullptr) != (fall_ps == nullptr)) return gs_fail(ctx, GS_E_INVALID, "give both wire arrays or neither");
    std::vector<int32_t> wr(d->F, 0), wf(d->F, 0);
    int32_t mx = 0;
    bool any = false;
    if (rise_ps) {
        for (int64_t s = 0; s < d->F; s++) {
            int32_t r = rise_ps[s], f = fall_ps[s];
            if (r < 0 || f < 0 || r > (1 << 24) || f > (1 << 24))
                return gs_fail(ctx, GS_E_INVALID, "wire %lld: delay out of range", (long long)s);
            if ((r == 0) != (f == 0))
                return gs_fail(ctx, GS_E_INVALID, "wire %lld: rise and fall must be both 0 or both >= 1", (long long)s);
            wr[s] = r;
            wf[s] = f;
            any = any || r > 0;
            mx = std::max(mx, std::max(r, f));
        }
    }
    if (any && d->arcs_loaded && d->zero_delay) return gs_fail(ctx, GS_E_INVALID, "zero-delay arcs need zero wire delays");
    d->wr.swap(wr);
    d->wf.swap(wf);
    d->has_wires = any;
    d->max_wire = mx;
    (void)hipSetDevice(ctx->opt.device);
    if (d->arcs_loaded) return pack_design(ctx, d);
    return GS_OK;
}

extern "C" gs_status gs_load_stimulus(gs_ctx *ctx, int32_t design, int32_t period_ps, int32_t n_cycles,
                                      const uint8_t *init, const int64_t *toggle_ptr, const int64_t *toggle_ps,
                                      int32_t *stim_id)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    gs_status st = check_stim_impl(ctx, d->I, period_ps, n_cycles, init, toggle_ptr, toggle_ps);
    if (st) return st;
    (void)hipSetDevice(ctx->opt.device);
    Stim *s = new Stim();
    s->design = design;
    s->period = period_ps;
    s->n_cycles = n_cycles;
    s->n_toggles = d->I ? toggle_ptr[d->I] : 0;
    void *p;
    if ((st = dev_alloc(ctx, &p, std::max(1, d->I)))) { delete s; return st; }
    s->d_init = (uint8_t *)p;
    if ((st = dev_alloc(ctx, &p, sizeof(int64_t) * (d->I + 1)))) { gs_dev_free(s->d_init); delete s; return st; }
    s->d_tp = (int64_t *)p;
    if ((st = dev_alloc(ctx, &p, sizeof(int64_t) * std::max<int64_t>(1, s->n_toggles)))) {
        gs_dev_free(s->d_init); gs_dev_free(s->d_tp); delete s; return st;
    }
    s->d_ts = (int64_t *)p;
    std::vector<int64_t> tp0(1, 0);
    const int64_t *tp = d->I ? toggle_ptr : tp0.data();
    hipStream_t hs = ctx->stream;
    if ((d->I && hipMemcpyAsync(s->d_init, init, d->I, hipMemcpyHostToDevice, hs) != hipSuccess) ||
        hipMemcpyAsync(s->d_tp, tp, sizeof(int64_t) * (d->I + 1), hipMemcpyHostToDevice, hs) != hipSuccess ||
        (s->n_toggles && hipMemcpyAsync(s->d_ts, toggle_ps, sizeof(int64_t) * s->n_toggles, hipMemcpyHostToDevice, hs) != hipSuccess) ||
        hipStreamSynchronize(hs) != hipSuccess) {
        gs_dev_free(s->d_init); gs_dev_free(s->d_tp); gs_dev_free(s->d_ts);
        delete s;
        return gs_fail(ctx, GS_E_DEVICE, "stimulus upload failed");
    }
    // toggles per cycle prefix (for window sizing)
    s->tog_prefix.assign((size_t)n_cycles + 1, 0);
    for (int32_t i = 0; i < d->I; i++)
        for (int64_t k = tp[i]; k < tp[i + 1]; k++) s->tog_prefix[toggle_ps[k] / period_ps + 1]++;
    for (int32_t c = 0; c < n_cycles; c++) s->tog_prefix[c + 1] += s->tog_prefix[c];
    ctx->stims.push_back(s);
    if (stim_id) *stim_id = (int32_t)ctx->stims.size() - 1;
    return GS_OK;
}

extern "C" gs_status gs_segment_stimulus(gs_ctx *ctx, int32_t stim, int32_t segment_cycles, int32_t *stim_id)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (stim < 0 || stim >= (int32_t)ctx->stims.size() || !ctx->stims[stim])
        return gs_fail(ctx, GS_E_INVALID, "no stimulus %d", stim);
    const Stim *s = ctx->stims[stim];
    if (s->carry) return gs_fail(ctx, GS_E_INVALID, "stimulus %d is a continuous view", stim);
    const int32_t S = segment_cycles;
    if (S < 1 || s->n_cycles % S)
        return gs_fail(ctx, GS_E_INVALID, "n_cycles %d is not a multiple of segment_cycles %d", s->n_cycles, S);
    if ((int64_t)s->period * S > (1 << 24))
        return gs_fail(ctx, GS_E_INVALID, "segment of %lld ps exceeds 2^24 ps", (long long)s->period * S);
    // a segment is a cycle of length S x period: the expansion, the walk
    // and the T0/T1 sums read nothing else
    Stim *v = new Stim();
    v->design = s->design;
    v->period = s->period * S;
    v->n_cycles = s->n_cycles / S;
    v->n_toggles = s->n_toggles;
    v->owns = false;
    v->d_init = s->d_init;
    v->d_tp = s->d_tp;
    v->d_ts = s->d_ts;
    v->tog_prefix.resize((size_t)v->n_cycles + 1);
    for (int32_t k = 0; k <= v->n_cycles; k++) v->tog_prefix[k] = s->tog_prefix[(size_t)k * S];
    ctx->stims.push_back(v);
    if (stim_id) *stim_id = (int32_t)ctx->stims.size() - 1;
    return GS_OK;
}

extern "C" gs_status gs_continuous_stimulus(gs_ctx *ctx, int32_t stim, int32_t segment_cycles, int32_t *stim_id)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (stim < 0 || stim >= (int32_t)ctx->stims.size() || !ctx->stims[stim])
        return gs_fail(ctx, GS_E_INVALID, "no stimulus %d", stim);
    const Stim *s = ctx->stims[stim];
    if (!s->owns || s->carry) return gs_fail(ctx, GS_E_INVALID, "stimulus %d is a view", stim);
    const int32_t S = segment_cycles;
    if (S < 1 || s->n_cycles % S)
        return gs_fail(ctx, GS_E_INVALID, "n_cycles %d is not a multiple of segment_cycles %d", s->n_cycles, S);
    // the cycles stay single cycles: the expansion, the lane lists and the
    // T0/T1 sums are those of the stimulus itself
    Stim *v = new Stim();
    v->design = s->design;
    v->period = s->period;
    v->n_cycles = s->n_cycles;
    v->n_toggles = s->n_toggles;
    v->owns = false;
    v->carry = S;
    v->d_init = s->d_init;
    v->d_tp = s->d_tp;
    v->d_ts = s->d_ts;
    v->tog_prefix = s->tog_prefix;
    ctx->stims.push_back(v);
    if (stim_id) *stim_id = (int32_t)ctx->stims.size() - 1;
    return GS_OK;
}

gs_status gs_job_cycles(gs_ctx *ctx, int32_t stim, int32_t &b, int32_t &e)
{
    if (stim < 0 || stim >= (int32_t)ctx->stims.size() || !ctx->stims[stim]) return GS_OK;   // reported by the caller
    const int32_t S = ctx->stims[stim]->carry;
    if (S <= 0) return GS_OK;
    const int64_t nseg = ctx->stims[stim]->n_cycles / S;
    if (b < 0 || e < b || e > nseg) return gs_fail(ctx, GS_E_INVALID, "segment range [%d, %d) outside [0, %lld)", b, e, (long long)nseg);
    b *= S;
    e *= S;
    return GS_OK;
}

// ---------------------------------------------------------------------------
// windows
// ---------------------------------------------------------------------------
void gs_window_release(gs_ctx *ctx, WindowBufs *w)
{
    if (!ctx->opt.arena) {
        gs_dev_free(w->hdr);
        gs_dev_free(w->ends);
        gs_dev_free(w->times);
    }
    *w = WindowBufs();
}

// Makes sure `w` holds at least n_chunks chunk headers and `words` arena words.
gs_status gs_window_reserve(gs_ctx *ctx, WindowBufs *w, uint64_t n_chunks, uint64_t words)
{
    if (ctx->opt.arena) {
        // carve [hdr | ends | times] out of the caller's arena
        uint64_t hb = (n_chunks * sizeof(ChunkHdr) + 255) & ~255ull;
        uint64_t eb = (n_chunks * kLanes * sizeof(uint16_t) + 255) & ~255ull;
        // the window gets all the space left after its headers and lane ends
        // (the planner's byte count leaves out the 256-byte alignment above)
        (void)words;
        if (hb + eb + (64ull << 10) > ctx->opt.arena_bytes)
            return gs_fail(ctx, GS_E_NOMEM, "arena too small for the window");
        char *base = (char *)ctx->opt.arena;
        w->hdr = (ChunkHdr *)base;
        w->ends = (uint16_t *)(base + hb);
        w->times = (int32_t *)(base + hb + eb);
        w->chunks = n_chunks;
        w->words = (ctx->opt.arena_bytes - hb - eb) / sizeof(int32_t);
        return GS_OK;
    }
    gs_status st;
    if (w->chunks < n_chunks) {
        gs_dev_free(w->hdr);
        gs_dev_free(w->ends);
        w->hdr = nullptr;
        w->ends = nullptr;
        w->chunks = 0;
        void *p;
        if ((st = dev_alloc(ctx, &p, n_chunks * sizeof(ChunkHdr)))) return st;
        w->hdr = (ChunkHdr *)p;
        if ((st = dev_alloc(ctx, &p, n_chunks * kLanes * sizeof(uint16_t)))) return st;
        w->ends = (uint16_t *)p;
        w->chunks = n_chunks;
    }
    if (w->words < words) {
        gs_dev_free(w->times);
        w->times = nullptr;
        w->words = 0;
        void *p;
        if ((st = dev_alloc(ctx, &p, words * sizeof(int32_t)))) return st;
        w->times = (int32_t *)p;
        w->words = words;
    }
    return GS_OK;
}

uint64_t gs_header_bytes(uint64_t n_nets, int32_t cycles)
{
    uint64_t tiles = (uint64_t)(cycles + kLanes - 1) / kLanes;
    return n_nets * tiles * (sizeof(ChunkHdr) + kLanes * sizeof(uint16_t));
}

// Initial arena size for a window: two words per (net, cycle) plus the
// window's input toggles, at least 16M words.
uint64_t gs_arena_guess(uint64_t n_nets, int32_t cycles, int64_t toggles)
{
    uint64_t w = n_nets * (uint64_t)cycles * 2ull + (uint64_t)toggles + (1ull << 20);
    return std::max<uint64_t>(w, 1ull << 24);
}

gs_status gs_check_ranges(gs_ctx *ctx, const Design *d, const Stim *s, int32_t b, int32_t e)
{
    if (!d->arcs_loaded) return gs_fail(ctx, GS_E_STATE, "load delay arcs before simulating");
    if (b < 0 || e < b || e > s->n_cycles) return gs_fail(ctx, GS_E_INVALID, "cycle range [%d, %d) outside [0, %d)", b, e, s->n_cycles);
    if (d->zero_delay && d->has_wires) return gs_fail(ctx, GS_E_INVALID, "zero-delay arcs need zero wire delays");
    if (s->carry && d->has_wires)
        return gs_fail(ctx, GS_E_INVALID, "continuous views run designs without interconnect delays");
    // every cycle-local time, including the latest possible edge, must fit int32
    const int64_t latest = (int64_t)s->period + (int64_t)(d->L + 1) * ((int64_t)d->max_delay + d->max_wire);
    if (latest >= (int64_t)kInf - 1) return gs_fail(ctx, GS_E_INVALID, "period + depth x delays exceeds int32 picoseconds");
    return GS_OK;
}

WinView gs_make_view(gs_ctx *ctx, const WindowBufs &w, int32_t cycles, int32_t period, uint64_t chunk_base,
                     uint64_t n_chunks_used)
{
    (void)n_chunks_used;
    WinView v;
    std::memset(&v, 0, sizeof(v));
    v.hdr = w.hdr + chunk_base;
    v.ends = w.ends + chunk_base * kLanes;
    v.times = w.times;
    // stripes: a power of two, each slice at least 4096 words
    uint32_t stripes = 1;
    while (stripes < (uint32_t)kMaxStripes && w.words / (2ull * stripes) >= 4096) stripes *= 2;
    v.bump = ctx->d_bump;
    v.flags = (unsigned int *)(ctx->d_misc + 1);
    v.slice_words = w.words / stripes;
    v.stripe_mask = stripes - 1;
    v.n_tiles = (cycles + kLanes - 1) / kLanes;
    v.n_cycles = cycles;
    v.period = period;
    return v;
}

gs_status gs_ensure_segs(gs_ctx *ctx, size_t n)
{
    if (ctx->segs_cap >= n) return GS_OK;
    gs_dev_free(ctx->d_segs);
    ctx->d_segs = nullptr;
    ctx->segs_cap = 0;
    void *p;
    gs_status st = dev_alloc(ctx, &p, sizeof(Seg) * std::max<size_t>(n, 64));
    if (st) return st;
    ctx->d_segs = (Seg *)p;
    ctx->segs_cap = std::max<size_t>(n, 64);
    return GS_OK;
}

hipEvent_t gs_event(gs_ctx *ctx, size_t i)
{
    while (ctx->events.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->events.push_back(e);
    }
    return ctx->events[i];
}

extern "C" gs_status gs_read_saif(gs_ctx *ctx, int32_t design, int64_t *tc, int64_t *t0, int64_t *t1, int32_t reset)
{
    return gs_read_saif_ig(ctx, design, tc, t0, t1, nullptr, reset);
}

extern "C" gs_status gs_read_saif_ig(gs_ctx *ctx, int32_t design, int64_t *tc, int64_t *t0, int64_t *t1, int64_t *ig,
                                     int32_t reset)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    (void)hipSetDevice(ctx->opt.device);
    hipStream_t hs = ctx->stream;
    const size_t n = (size_t)d->N;
    if (n) {
        if (tc) HIPCHK(hipMemcpyAsync(tc, d->d_saif, n * 8, hipMemcpyDeviceToHost, hs));
        if (t0) HIPCHK(hipMemcpyAsync(t0, d->d_saif + n, n * 8, hipMemcpyDeviceToHost, hs));
        if (t1) HIPCHK(hipMemcpyAsync(t1, d->d_saif + 2 * n, n * 8, hipMemcpyDeviceToHost, hs));
        if (ig) HIPCHK(hipMemcpyAsync(ig, d->d_saif + 3 * n, n * 8, hipMemcpyDeviceToHost, hs));
        if (reset) HIPCHK(launch_fill_u64(d->d_saif, kSaifArrays * n, 0ull, hs));
    }
    HIPCHK(hipStreamSynchronize(hs));
    return GS_OK;
}

extern "C" gs_status gs_read_waveform(gs_ctx *ctx, int32_t design, int32_t stim, int32_t net, int32_t cycle,
                                      int32_t *init, int32_t *times, int32_t cap, int32_t *n)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    if (net < 0 || net >= d->N) return gs_fail(ctx, GS_E_INVALID, "net %d out of range", net);
    // a continuous view's segment is the concatenation of its cycles' lists
    const Stim *sv = (stim >= 0 && stim < (int32_t)ctx->stims.size()) ? ctx->stims[stim] : nullptr;
    const int32_t S = sv && sv->carry > 0 ? sv->carry : 1;
    const int64_t c_first = (int64_t)cycle * S;
    const LastWindow *found = nullptr;
    for (const LastWindow &w : ctx->last)
        if (w.design == design && w.stim == stim && cycle >= 0 && c_first >= w.c0 && c_first + S <= (int64_t)w.c0 + w.cycles)
            found = &w;
    if (!found && ctx->last_released)
        return gs_fail(ctx, GS_E_STATE, "waveforms are not kept when dead nets are released (gs_options.release_dead)");
    if (!found) return gs_fail(ctx, GS_E_STATE, "cycle %d of (design %d, stim %d) is not resident", cycle, design, stim);
    const LastWindow &lw = *found;
    if (S > 1 && (int64_t)S * sv->period + (int64_t)(d->L + 1) * d->max_delay >= (int64_t)kInf)
        return gs_fail(ctx, GS_E_INVALID, "segment times exceed int32 picoseconds");
    (void)hipSetDevice(ctx->opt.device);
    hipStream_t hs = ctx->stream;
    const int32_t tiles = (lw.cycles + kLanes - 1) / kLanes;
    int64_t total = 0;
    for (int32_t k = 0; k < S; k++) {
        const int32_t local = (int32_t)(c_first - lw.c0) + k;
        const int32_t tile = local / kLanes, lane = local % kLanes;
        const uint64_t ci = lw.chunk_base + (uint64_t)net * tiles + tile;
        ChunkHdr h;
        uint16_t e[kLanes];
        HIPCHK(hipMemcpyAsync(&h, ctx->win.hdr + ci, sizeof(h), hipMemcpyDeviceToHost, hs));
        HIPCHK(hipMemcpyAsync(e, ctx->win.ends + ci * kLanes, sizeof(e), hipMemcpyDeviceToHost, hs));
        HIPCHK(hipStreamSynchronize(hs));
        const uint32_t lo = lane ? e[lane - 1] & kEndCount : 0, hi = e[lane] & kEndCount;
        if (k == 0 && init) *init = (int32_t)((h.mask >> lane) & 1);
        const int64_t room = cap > 0 ? (int64_t)cap - total : 0;
        const uint32_t m = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(hi - lo, room));
        if (m && times) {
            int32_t *dst = times + total;
            HIPCHK(hipMemcpyAsync(dst, ctx->win.times + h.off + lo, sizeof(int32_t) * m, hipMemcpyDeviceToHost, hs));
            HIPCHK(hipStreamSynchronize(hs));
            for (uint32_t i = 0; i < m; i++) dst[i] += k * sv->period;
        }
        total += hi - lo;
    }
    if (n) *n = (int32_t)std::min<int64_t>(total, INT32_MAX);
    return GS_OK;
}

extern "C" gs_status gs_get_design_info(gs_ctx *ctx, int32_t design, gs_design_info *info)
{
    if (!ctx || !info) return gs_fail(ctx, GS_E_INVALID, "null argument");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    std::memset(info, 0, sizeof(*info));
    info->n_inputs = d->I;
    info->n_gates = d->G;
    info->n_levels = d->L;
    info->max_pins = d->max_pins;
    info->n_fanin = d->F;
    info->has_wires = d->has_wires;
    info->zero_delay = d->zero_delay;
    info->max_delay_ps = d->max_delay;
    return GS_OK;
}

extern "C" gs_status gs_get_levels(gs_ctx *ctx, int32_t design, int32_t *level)
{
    if (!ctx || !level) return gs_fail(ctx, GS_E_INVALID, "null argument");
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    std::memcpy(level, d->level.data(), sizeof(int32_t) * d->G);
    return GS_OK;
}

extern "C" gs_status gs_get_stats(gs_ctx *ctx, gs_stats *st, int32_t reset)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (st) *st = ctx->stats;
    if (reset) std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    return GS_OK;
}
