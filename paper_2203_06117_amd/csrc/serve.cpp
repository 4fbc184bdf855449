// Serving: a resident request loop with continuous batching.
//
// The re-simulation step of GATSPI's glitch-optimization flow (Section 4)
// as a service: netlists stay on the device, requests are either a new
// stimulus window or a set of delay edits whose fanout cone is re-simulated
// against a resident window.  A scheduler thread admits queued requests
// while their device-memory footprint fits the free pool, and every step
// launches the next level of every request in flight in one launch, so a
// request admitted while others run joins the schedule at once.
#include "host.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <vector>

using namespace gs;

namespace {

constexpr int kRing = 64;               // segment tables in flight
constexpr int kPinned = 16;             // pinned result buffers

enum State { Q_WAIT = 0, Q_ADMITTED = 1, Q_RUN = 2, Q_FINAL = 3, Q_DONE = 4 };

struct Region {
    uint64_t off = 0, bytes = 0;
};

// First-fit allocator over one device buffer (offsets, 256-byte aligned).
struct Pool {
    char *base = nullptr;
    uint64_t bytes = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> size

    void init(char *b, uint64_t n)
    {
        base = b;
        bytes = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(uint64_t n, Region &r)
    {
        n = (n + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            r.off = it->first;
            r.bytes = n;
            const uint64_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(const Region &r)
    {
        if (!r.bytes) return;
        auto it = free_.emplace(r.off, r.bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t largest() const
    {
        uint64_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

struct Resident {
    int32_t design, stim, c0, cycles, tiles;
    Region region;
    ChunkHdr *hdr;
    uint16_t *ends;
    unsigned long long *saif;            // SAIF accumulators of the resident window (SaifAcc order)
};

struct Req {
    uint64_t ticket = 0;
    gs_request r{};
    std::vector<gs_arc_edit> edits;
    int state = Q_WAIT;
    gs_status status = GS_OK;
    std::string err;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<int64_t> tc, t0, t1, ig;
    int64_t gate_cycles = 0;
    // execution
    Design *d = nullptr;
    Stim *s = nullptr;
    int32_t res_idx = -1;
    int32_t c0 = 0, cycles = 0, tiles = 0;
    Region region;
    uint64_t arena_words = 0;
    int attempts = 0;
    WinView view{};
    SaifAcc acc{};
    unsigned long long *bump = nullptr;
    unsigned int *flags = nullptr;
    int32_t *d_c0 = nullptr;
    const GateRec *gates = nullptr;
    const PinRec *pins = nullptr;
    std::vector<uint32_t> lvl_begin, lvl_n;   // per level 1..L (index l-1): gates of the level
    size_t next = 0;                          // index into lvl_* of the next level to launch
    uint32_t n_cone = 0;
    int pinned = -1;
    hipEvent_t ev = nullptr;
    // delay edits: cone preparation scratch (marks, per-level counts and
    // offsets, net -> cone slot, edited records)
    Region prep;
    uint8_t *d_mark = nullptr;
    unsigned int *d_cnt = nullptr, *d_cur = nullptr, *d_off = nullptr;
    int32_t *d_slot = nullptr;
    EditRec *d_edits = nullptr;
    uint32_t *d_enets = nullptr;
    uint32_t stride = 1;
    hipEvent_t ev_prep = nullptr;
};

using ReqP = std::shared_ptr<Req>;

}  // namespace

struct ServeState {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    bool stop = false;
    int32_t max_queue = 0;
    uint64_t next_ticket = 1;
    std::deque<ReqP> queue;
    std::map<uint64_t, ReqP> all;
    std::vector<ReqP> active, finalizing;
    std::vector<Resident> res;
    hipStream_t st = nullptr, prep = nullptr;
    Pool pool;
    void *pool_ptr = nullptr;
    Seg *seg_ring = nullptr;
    size_t seg_cap = 0;
    hipEvent_t ring_ev[kRing] = {};
    int ring_pos = 0;
    void *pinned[kPinned] = {};
    uint64_t pinned_bytes = 0;
    bool pinned_busy[kPinned] = {};
    Seg *h_seg_ring = nullptr;                          // pinned staging of the segment tables
    char *h_small = nullptr;                            // pinned staging of edit records and level offsets
    std::map<Design *, double> words_per_net_cycle;   // observed arena need
    uint64_t salt = 0;
    gs_status fatal = GS_OK;
    std::string fatal_msg;
};

namespace {

#define SCHK(x)                                                                              \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) {                                                              \
            err = std::string(#x) + ": " + hipGetErrorString(e_);                            \
            return GS_E_DEVICE;                                                              \
        }                                                                                    \
    } while (0)

template <typename T>
T *at(ServeState *S, uint64_t off)
{
    return (T *)(S->pool.base + off);
}

uint64_t align256(uint64_t x)
{
    return (x + 255) & ~255ull;
}

// Footprint of a request's region: chunk headers and lane ends for `rows`
// nets, the transition arena, SAIF staging, stripe counters and flags, and
// for edits the cone's remap, gate and pin records.
uint64_t region_bytes(uint64_t rows, int32_t tiles, uint64_t words, uint64_t n_nets, uint64_t cone_gates,
                      uint64_t cone_pins, bool edit)
{
    uint64_t b = 0;
    b += align256(rows * tiles * sizeof(ChunkHdr));
    b += align256(rows * tiles * kLanes * sizeof(uint16_t));
    b += align256(words * sizeof(int32_t));
    b += align256(kSaifArrays * n_nets * sizeof(unsigned long long));
    b += align256((uint64_t)kMaxStripes * kBumpStride * sizeof(unsigned long long));
    b += 256;                                               // flags + first cycle
    if (edit) {
        b += align256(cone_gates * sizeof(GateRec));
        b += align256(cone_pins * sizeof(PinRec));
    }
    return b;
}

// Lays the request's views out over its region.
void layout(ServeState *S, Req &q, uint64_t rows)
{
    uint64_t o = q.region.off;
    ChunkHdr *hdr = at<ChunkHdr>(S, o);
    o += align256(rows * q.tiles * sizeof(ChunkHdr));
    uint16_t *ends = at<uint16_t>(S, o);
    o += align256(rows * q.tiles * kLanes * sizeof(uint16_t));
    const uint64_t arena_off_bytes = o;
    o += align256(q.arena_words * sizeof(int32_t));
    unsigned long long *saif = at<unsigned long long>(S, o);
    o += align256(kSaifArrays * (uint64_t)q.d->N * sizeof(unsigned long long));
    q.bump = at<unsigned long long>(S, o);
    o += align256((uint64_t)kMaxStripes * kBumpStride * sizeof(unsigned long long));
    q.flags = at<unsigned int>(S, o);
    q.d_c0 = (int32_t *)(S->pool.base + o + 64);
    o += 256;
    std::memset(&q.view, 0, sizeof(q.view));
    q.view.hdr = hdr;
    q.view.ends = ends;
    q.view.times = (int32_t *)S->pool.base;
    q.view.bump = q.bump;
    q.view.flags = q.flags;
    uint32_t stripes = 1;
    while (stripes < (uint32_t)kMaxStripes && q.arena_words / (2ull * stripes) >= 4096) stripes *= 2;
    q.view.slice_words = q.arena_words / stripes;
    q.view.stripe_mask = stripes - 1;
    q.view.arena_off = arena_off_bytes / sizeof(int32_t);
    q.view.n_tiles = q.tiles;
    q.view.n_cycles = q.cycles;
    q.view.period = q.s->period;
    q.acc = saif_view(saif, (size_t)q.d->N);
    if (q.r.kind == GS_REQ_EDIT) {
        GateRec *g = at<GateRec>(S, o);
        o += align256((uint64_t)q.n_cone * sizeof(GateRec));
        q.view.slot = q.d_slot;
        q.view.rd_hdr = S->res[q.res_idx].hdr;
        q.view.rd_ends = S->res[q.res_idx].ends;
        q.gates = g;
        q.pins = at<PinRec>(S, o);
    } else {
        q.gates = q.d->d_gates;
        q.pins = q.d->d_pins;
    }
}

uint64_t guess_words(ServeState *S, Design *d, uint64_t rows, int32_t cycles, int64_t toggles)
{
    double w = 1.0;
    auto it = S->words_per_net_cycle.find(d);
    if (it != S->words_per_net_cycle.end()) w = std::max(0.05, it->second * 1.25);
    return std::max<uint64_t>((uint64_t)(w * (double)rows * cycles) + (uint64_t)toggles + (1ull << 16), 1ull << 20);
}

// Device-side preparation of an admitted request on the execution stream.
gs_status start_request(gs_ctx *ctx, ServeState *S, Req &q, std::string &err)
{
    hipStream_t hs = S->st;
    SCHK(launch_fill_u32(q.flags, 16, 0u, hs));
    SCHK(launch_fill_u64(q.bump, (uint64_t)kMaxStripes * kBumpStride, 0ull, hs));
    if (q.r.kind == GS_REQ_WINDOW) {
        SCHK(launch_fill_u64(q.acc.tc, kSaifArrays * (uint64_t)q.d->N, 0ull, hs));
        SCHK(launch_fill_u32((unsigned int *)q.d_c0, 1, (unsigned int)q.c0, hs));
        StimView sv{q.s->d_init, q.s->d_tp, q.s->d_ts, q.d->I, q.s->period, 0};
        SCHK(launch_expand(sv, q.view, q.acc, q.d_c0, (uint32_t)(S->salt++ * 131), hs));
    } else {
        const Resident &R = S->res[q.res_idx];
        SCHK(hipStreamWaitEvent(hs, q.ev_prep, 0));
        SCHK(hipMemcpyAsync(q.acc.tc, R.saif, kSaifArrays * sizeof(unsigned long long) * q.d->N, hipMemcpyDeviceToDevice,
                            hs));
        SCHK(launch_saif_zero(q.gates, q.n_cone, q.acc, hs));
    }
    (void)ctx;
    return GS_OK;
}

// Host part of admission: region sizing and allocation, edits applied,
// fanout cone marked on the device and its records uploaded.
gs_status admit(gs_ctx *ctx, ServeState *S, Req &q, bool &fits, std::string &err)
{
    fits = true;
    Design *d = q.d;
    if (q.r.kind == GS_REQ_WINDOW) {
        q.c0 = q.r.cycle_begin;
        q.cycles = q.r.cycle_end - q.r.cycle_begin;
        q.tiles = (q.cycles + kLanes - 1) / kLanes;
        if (!q.arena_words)
            q.arena_words = guess_words(S, d, (uint64_t)d->N, q.cycles,
                                        q.s->tog_prefix[q.c0 + q.cycles] - q.s->tog_prefix[q.c0]);
        const uint64_t need = region_bytes(d->N, q.tiles, q.arena_words, d->N, 0, 0, false);
        if (need > S->pool.bytes) {
            err = "request does not fit the serving pool";
            return GS_E_NOMEM;
        }
        if (!S->pool.alloc(need, q.region)) {
            fits = false;
            return GS_OK;
        }
        layout(S, q, d->N);
        q.lvl_begin.clear();
        q.lvl_n.clear();
        for (int32_t l = 1; l <= d->L; l++) {
            q.lvl_begin.push_back(d->level_ptr[l]);
            q.lvl_n.push_back(d->level_ptr[l + 1] - d->level_ptr[l]);
        }
        q.gate_cycles = (int64_t)d->G * q.cycles;
        return GS_OK;
    }
    // delay edit: new delays per touched fanin slot, computed from the
    // slot's arc records with the edited records substituted
    const Resident &R = S->res[q.res_idx];
    q.c0 = R.c0;
    q.cycles = R.cycles;
    q.tiles = R.tiles;
    std::map<int64_t, std::array<int32_t, 2>> newdel;     // arc record -> (rise, fall)
    std::map<int64_t, int32_t> slots;                     // touched fanin slot -> gate
    for (const gs_arc_edit &e : q.edits) {
        if (e.gate < 0 || e.gate >= d->G || e.pin < 0 || e.pin >= d->gate_k[e.gate]) {
            err = "edit names a pin that does not exist";
            return GS_E_INVALID;
        }
        const int64_t sl = d->fanin_ptr[e.gate] + e.pin;
        if (e.in_edge < 0 || e.in_edge > 2) {
            err = "edit has a bad input-edge qualifier";
            return GS_E_INVALID;
        }
        const int64_t a = d->slot_rec[kArcKinds * sl + arc_kind(e)];
        if (a == -2) {
            err = "edit names more than one arc record";
            return GS_E_INVALID;
        }
        if (a < 0 || (e.cond_pin >= 0 && d->arcs[a].cond_pin != e.cond_pin)) {
            err = "edit names an arc record that does not exist";
            return GS_E_INVALID;
        }
        const bool zero = d->zero_delay != 0;
        if (e.rise_ps < 0 || e.fall_ps < 0 || e.rise_ps > (1 << 24) || e.fall_ps > (1 << 24) ||
            (!zero && (e.rise_ps < 1 || e.fall_ps < 1)) || (zero && (e.rise_ps || e.fall_ps))) {
            err = "edited delay out of range";
            return GS_E_INVALID;
        }
        newdel[a] = {e.rise_ps, e.fall_ps};
        slots[sl] = e.gate;
    }
    if (slots.size() > 65536) {
        err = "at most 65536 edited pins per request";
        return GS_E_INVALID;
    }
    std::vector<EditRec> er;
    std::vector<uint32_t> enets;
    for (auto &kv : slots) {
        const int64_t sl = kv.first;
        const int32_t g = kv.second;
        auto del = [&](int64_t a, int rise) -> int32_t {
            auto it = newdel.find(a);
            if (it != newdel.end()) return it->second[rise ? 0 : 1];
            return rise ? d->arcs[a].rise_ps : d->arcs[a].fall_ps;
        };
        EditRec e;
        e.out = (uint32_t)(d->I + g);
        e.pin = (uint32_t)(sl - d->fanin_ptr[g]);
        for (int cv = 0; cv < 2; cv++)
            for (int ie = 0; ie < 2; ie++) {
                // the load resolved every combination, so a unique winner exists
                const int64_t w = arc_winner(&d->slot_rec[kArcKinds * sl], cv, ie);
                e.d[gs::delay_slot(cv, ie, 1)] = del(w, 1);
                e.d[gs::delay_slot(cv, ie, 0)] = del(w, 0);
            }
        er.push_back(e);
        if (enets.empty() || enets.back() != e.out) enets.push_back(e.out);
    }
    // preparation scratch: marks, counts, cursors, offsets, slots, edit records
    const uint64_t L2 = (uint64_t)d->L + 2;
    uint64_t pb = 0;
    const uint64_t o_mark = pb;  pb += align256(d->N);
    const uint64_t o_cnt = pb;   pb += align256(L2 * 4);
    const uint64_t o_cur = pb;   pb += align256(L2 * 4);
    const uint64_t o_off = pb;   pb += align256(L2 * 4);
    const uint64_t o_slot = pb;  pb += align256((uint64_t)d->N * 4);
    const uint64_t o_ed = pb;    pb += align256(er.size() * sizeof(EditRec));
    const uint64_t o_en = pb;    pb += align256(enets.size() * 4);
    if (!q.prep.bytes) {
        if (!S->pool.alloc(pb, q.prep)) {
            fits = false;
            return GS_OK;
        }
    }
    q.d_mark = at<uint8_t>(S, q.prep.off + o_mark);
    q.d_cnt = at<unsigned int>(S, q.prep.off + o_cnt);
    q.d_cur = at<unsigned int>(S, q.prep.off + o_cur);
    q.d_off = at<unsigned int>(S, q.prep.off + o_off);
    q.d_slot = at<int32_t>(S, q.prep.off + o_slot);
    q.d_edits = at<EditRec>(S, q.prep.off + o_ed);
    q.d_enets = at<uint32_t>(S, q.prep.off + o_en);
    // mark the fanout cone level by level on the preparation stream and
    // read back the per-level cone sizes (the only host wait of an edit)
    hipStream_t ps = S->prep;
    char *h_ed = S->h_small, *h_off = S->h_small + (2u << 20);
    std::memcpy(h_ed, er.data(), er.size() * sizeof(EditRec));
    std::memcpy(h_ed + (1u << 20) + (512u << 10), enets.data(), enets.size() * 4);
    hipError_t he = launch_fill_u32((unsigned int *)q.d_mark, (d->N + 3) / 4, 0u, ps);
    if (he == hipSuccess) he = launch_fill_u32(q.d_cnt, L2, 0u, ps);
    if (he == hipSuccess) he = launch_fill_u32(q.d_cur, L2, 0u, ps);
    if (he == hipSuccess) he = launch_fill_u32((unsigned int *)q.d_slot, d->N, 0xffffffffu, ps);
    if (he == hipSuccess) he = hipMemcpyAsync(q.d_edits, h_ed, er.size() * sizeof(EditRec), hipMemcpyHostToDevice, ps);
    if (he == hipSuccess)
        he = hipMemcpyAsync(q.d_enets, h_ed + (1u << 20) + (512u << 10), enets.size() * 4, hipMemcpyHostToDevice, ps);
    if (he == hipSuccess) he = launch_mark_set(q.d_enets, (uint32_t)enets.size(), q.d_mark, ps);
    for (int32_t l = 1; l <= d->L && he == hipSuccess; l++)
        he = launch_cone_mark(d->d_gates, d->d_pins, d->level_ptr[l], d->level_ptr[l + 1] - d->level_ptr[l], q.d_mark,
                              q.d_cnt + l, ps);
    std::vector<unsigned int> cnt(L2, 0);
    if (he == hipSuccess) he = hipMemcpyAsync(h_off, q.d_cnt, L2 * 4, hipMemcpyDeviceToHost, ps);
    if (he == hipSuccess) he = hipStreamSynchronize(ps);
    if (he != hipSuccess) {
        err = std::string("cone marking: ") + hipGetErrorString(he);
        return GS_E_DEVICE;
    }
    std::memcpy(cnt.data(), h_off, L2 * 4);
    std::vector<unsigned int> off(L2, 0);
    q.lvl_begin.clear();
    q.lvl_n.clear();
    uint32_t total = 0;
    for (int32_t l = 1; l <= d->L; l++) {
        off[l] = total;
        q.lvl_begin.push_back(total);
        q.lvl_n.push_back(cnt[l]);
        total += cnt[l];
    }
    off[d->L + 1] = total;
    q.n_cone = total;
    q.stride = (uint32_t)std::max(1, d->max_pins);
    if (!q.arena_words) q.arena_words = guess_words(S, d, std::max<uint32_t>(q.n_cone, 1), q.cycles, 0);
    const uint64_t need = region_bytes(std::max<uint32_t>(q.n_cone, 1), q.tiles, q.arena_words, d->N, q.n_cone,
                                       (uint64_t)q.n_cone * q.stride, true);
    if (need > S->pool.bytes) {
        err = "request does not fit the serving pool";
        return GS_E_NOMEM;
    }
    if (!S->pool.alloc(need, q.region)) {
        fits = false;                      // keeps its preparation region; marking is redone on retry
        return GS_OK;
    }
    layout(S, q, std::max<uint32_t>(q.n_cone, 1));
    // place the cone's records and apply the edits, still on the preparation stream
    std::memcpy(h_off, off.data(), L2 * 4);
    he = hipMemcpyAsync(q.d_off, h_off, L2 * 4, hipMemcpyHostToDevice, ps);
    if (he == hipSuccess)
        he = launch_cone_place(d->d_gates, d->d_pins, (uint32_t)d->G, q.d_mark, d->d_level, q.d_off, q.d_cur,
                               (GateRec *)q.gates, (PinRec *)q.pins, q.stride, q.d_slot, q.n_cone, ps);
    if (he == hipSuccess)
        he = launch_edit_apply(q.d_edits, (uint32_t)er.size(), q.d_slot, (PinRec *)q.pins, q.stride, q.n_cone, ps);
    if (he == hipSuccess && !q.ev_prep) he = hipEventCreateWithFlags(&q.ev_prep, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventRecord(q.ev_prep, ps);
    if (he != hipSuccess) {
        S->pool.release(q.region);
        q.region = Region();
        err = std::string("cone placement: ") + hipGetErrorString(he);
        return GS_E_DEVICE;
    }
    q.gate_cycles = (int64_t)q.n_cone * q.cycles;
    (void)ctx;
    return GS_OK;
}

int take_pinned(ServeState *S)
{
    for (int i = 0; i < kPinned; i++)
        if (!S->pinned_busy[i]) {
            S->pinned_busy[i] = true;
            return i;
        }
    return -1;
}

// One scheduler iteration's device step: the next level of every running
// request, gathered into one launch per kernel kind (plain, cone remap).
gs_status launch_step(gs_ctx *ctx, ServeState *S, std::vector<ReqP> &run, std::string &err)
{
    std::vector<Seg> segs[2];
    uint64_t waves[2] = {0, 0};
    int32_t kmax[2] = {1, 1}, wires[2] = {0, 0};
    const uint32_t tpw = (uint32_t)ctx->opt.tiles_per_wave, wpb = (uint32_t)ctx->opt.waves_per_block;
    for (ReqP &q : run) {
        // skip levels without gates (cones are sparse)
        while (q->next < q->lvl_n.size() && q->lvl_n[q->next] == 0) q->next++;
        if (q->next >= q->lvl_n.size()) continue;
        const int kind = q->r.kind == GS_REQ_EDIT ? 1 : 0;
        const int32_t l = (int32_t)q->next + 1;
        Seg g;
        std::memset(&g, 0, sizeof(g));
        const uint64_t ngroup = ((uint64_t)q->tiles + tpw - 1) / tpw;
        g.wave_begin = waves[kind];
        g.gates = q->gates;
        g.pins = q->pins;
        g.gate_begin = q->lvl_begin[q->next];
        g.n_gates = q->lvl_n[q->next];
        g.salt = (uint32_t)S->salt;
        g.mode = ctx->opt.wire_transport ? 1u : 0u;
        g.win = q->view;
        g.saif = q->acc;
        const uint64_t nw = (uint64_t)g.n_gates * ngroup;
        waves[kind] += nw;
        S->salt += (nw + wpb - 1) / wpb * tpw;
        kmax[kind] = std::max(kmax[kind], q->d->level_kmax[l]);
        wires[kind] |= q->d->has_wires ? 1 : 0;
        segs[kind].push_back(g);
        q->next++;
    }
    for (int kind = 0; kind < 2; kind++) {
        if (segs[kind].empty()) continue;
        const int slot = S->ring_pos;
        S->ring_pos = (S->ring_pos + 1) % kRing;
        SCHK(hipEventSynchronize(S->ring_ev[slot]));       // the table's previous use has finished
        if (segs[kind].size() > S->seg_cap) {
            err = "too many requests in one step";
            return GS_E_STATE;
        }
        Seg *dst = S->seg_ring + (size_t)slot * S->seg_cap;
        Seg *stage = S->h_seg_ring + (size_t)slot * S->seg_cap;
        std::memcpy(stage, segs[kind].data(), sizeof(Seg) * segs[kind].size());
        SCHK(hipMemcpyAsync(dst, stage, sizeof(Seg) * segs[kind].size(), hipMemcpyHostToDevice, S->st));
        SCHK(launch_gate_eval(dst, (int32_t)segs[kind].size(), waves[kind], wires[kind], ctx->opt.lds_cap,
                              ctx->opt.waves_per_block, kmax[kind], tpw, kind, 0, S->st));
        SCHK(hipEventRecord(S->ring_ev[slot], S->st));
    }
    return GS_OK;
}

void finish(ServeState *S, Req &q, gs_status st, const std::string &msg)
{
    q.status = st;
    q.err = msg;
    q.t_done = gs_now_ns();
    q.state = Q_DONE;
    if (q.region.bytes) S->pool.release(q.region);
    q.region = Region();
    if (q.prep.bytes) S->pool.release(q.prep);
    q.prep = Region();
    if (q.ev_prep) (void)hipEventDestroy(q.ev_prep);
    q.ev_prep = nullptr;
    if (q.pinned >= 0) S->pinned_busy[q.pinned] = false;
    q.pinned = -1;
    if (q.ev) (void)hipEventDestroy(q.ev);
    q.ev = nullptr;
}

void serve_loop(gs_ctx *ctx, ServeState *S)
{
    (void)hipSetDevice(ctx->opt.device);
    std::string err;
    for (;;) {
        std::vector<ReqP> fresh;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) break;
            if (S->queue.empty() && S->active.empty() && S->finalizing.empty())
                S->cv.wait_for(lk, std::chrono::milliseconds(50));
            if (S->stop) break;
            // admission in arrival order while the footprint fits
            while (!S->queue.empty()) {
                ReqP q = S->queue.front();
                bool fits = true;
                gs_status st = admit(ctx, S, *q, fits, err);
                if (st) {
                    S->queue.pop_front();
                    finish(S, *q, st, err);
                    S->cv_done.notify_all();
                    continue;
                }
                if (!fits) {
                    if (S->active.empty() && S->finalizing.empty() && fresh.empty()) {
                        // nothing will free up: the pool cannot hold this request
                        S->queue.pop_front();
                        finish(S, *q, GS_E_NOMEM, "request does not fit the free serving pool");
                        S->cv_done.notify_all();
                        continue;
                    }
                    break;
                }
                S->queue.pop_front();
                q->state = Q_RUN;
                q->t_admit = gs_now_ns();
                q->next = 0;
                fresh.push_back(q);
            }
        }
        gs_status st = GS_OK;
        for (ReqP &q : fresh) {
            st = start_request(ctx, S, *q, err);
            if (st) break;
            S->active.push_back(q);
        }
        if (!st && !S->active.empty()) st = launch_step(ctx, S, S->active, err);
        if (st) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->fatal = st;
            S->fatal_msg = err;
            for (ReqP &q : S->active) finish(S, *q, st, err);
            for (ReqP &q : S->finalizing) finish(S, *q, st, err);
            S->active.clear();
            S->finalizing.clear();
            S->cv_done.notify_all();
            break;
        }
        // requests past their last level: copy the SAIF staging and flags out
        for (size_t i = 0; i < S->active.size();) {
            ReqP q = S->active[i];
            while (q->next < q->lvl_n.size() && q->lvl_n[q->next] == 0) q->next++;
            if (q->next < q->lvl_n.size()) {
                i++;
                continue;
            }
            const int pb = take_pinned(S);
            if (pb < 0) break;                             // a buffer frees up once a finalize completes
            q->pinned = pb;
            char *h = (char *)S->pinned[pb];
            const size_t n3 = kSaifArrays * sizeof(unsigned long long) * q->d->N;
            hipError_t e = hipMemcpyAsync(h, q->acc.tc, n3, hipMemcpyDeviceToHost, S->st);
            if (e == hipSuccess) e = hipMemcpyAsync(h + n3, q->flags, 16, hipMemcpyDeviceToHost, S->st);
            if (e == hipSuccess) e = hipMemcpyAsync(h + n3 + 16, q->bump, sizeof(unsigned long long) * kMaxStripes * kBumpStride,
                                                    hipMemcpyDeviceToHost, S->st);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(q->ev, S->st);
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(S->mu);
                finish(S, *q, GS_E_DEVICE, hipGetErrorString(e));
                S->cv_done.notify_all();
            } else {
                q->state = Q_FINAL;
                S->finalizing.push_back(q);
            }
            S->active.erase(S->active.begin() + i);
        }
        // completed finalizations
        for (size_t i = 0; i < S->finalizing.size();) {
            ReqP q = S->finalizing[i];
            const bool idle = S->active.empty();
            hipError_t e = idle ? hipEventSynchronize(q->ev) : hipEventQuery(q->ev);
            if (e == hipErrorNotReady) {
                i++;
                continue;
            }
            // results are copied out of the pinned buffer before taking the lock
            const char *h = (const char *)S->pinned[q->pinned];
            const size_t N = (size_t)q->d->N;
            const unsigned int *fl = (const unsigned int *)(h + kSaifArrays * 8 * N);
            const unsigned long long *hb = (const unsigned long long *)(h + kSaifArrays * 8 * N + 16);
            const bool good = e == hipSuccess && !fl[0] && !fl[1] && !fl[3];
            if (good) {
                q->tc.resize(N);
                q->t0.resize(N);
                q->t1.resize(N);
                q->ig.resize(N);
                const unsigned long long *a = (const unsigned long long *)h;
                std::memcpy(q->tc.data(), a, 8 * N);
                std::memcpy(q->t0.data(), a + N, 8 * N);
                std::memcpy(q->t1.data(), a + 2 * N, 8 * N);
                std::memcpy(q->ig.data(), a + 3 * N, 8 * N);
            }
            std::lock_guard<std::mutex> lk(S->mu);
            if (e != hipSuccess) {
                finish(S, *q, GS_E_DEVICE, hipGetErrorString(e));
            } else if (fl[3]) {
                finish(S, *q, GS_E_DEVICE, "internal error: an output chunk exceeded its fanin bound");
            } else if (fl[1]) {
                finish(S, *q, GS_E_CAPACITY, "more than 32767 transitions in one (net, 64-cycle tile)");
            } else if (fl[0]) {
                // the arena filled up: run the request again with twice the arena
                S->pool.release(q->region);
                q->region = Region();
                S->pinned_busy[q->pinned] = false;
                q->pinned = -1;
                (void)hipEventDestroy(q->ev);
                q->ev = nullptr;
                q->arena_words *= 2;
                q->attempts++;
                q->state = Q_WAIT;
                S->queue.push_front(q);
            } else {
                uint64_t used = 0;
                for (uint32_t st2 = 0; st2 <= q->view.stripe_mask; st2++)
                    used += std::min<uint64_t>(hb[(size_t)st2 * kBumpStride] - hb[(size_t)st2 * kBumpStride + 1],
                                               q->view.slice_words);
                const double rows = q->r.kind == GS_REQ_EDIT ? std::max<uint32_t>(q->n_cone, 1) : q->d->N;
                const double wpc = (double)used / (rows * q->cycles);
                double &est = S->words_per_net_cycle[q->d];
                est = std::max(est * 0.9, wpc);
                finish(S, *q, GS_OK, "");
            }
            S->finalizing.erase(S->finalizing.begin() + i);
            S->cv_done.notify_all();
        }
    }
}

ServeState *serve_of(gs_ctx *ctx)
{
    return ctx ? ctx->serve : nullptr;
}

}  // namespace

void gs_serve_shutdown(gs_ctx *ctx)
{
    ServeState *S = serve_of(ctx);
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    if (S->st) (void)hipStreamSynchronize(S->st);
    for (auto &kv : S->all) {
        Req &q = *kv.second;
        if (q.state != Q_DONE) finish(S, q, GS_E_STATE, "serving stopped");
    }
    for (int i = 0; i < kRing; i++)
        if (S->ring_ev[i]) (void)hipEventDestroy(S->ring_ev[i]);
    for (int i = 0; i < kPinned; i++)
        if (S->pinned[i]) (void)hipHostFree(S->pinned[i]);
    gs_dev_free(S->seg_ring);
    if (S->h_seg_ring) (void)hipHostFree(S->h_seg_ring);
    if (S->h_small) (void)hipHostFree(S->h_small);
    gs_dev_free(S->pool_ptr);
    if (S->st) (void)hipStreamDestroy(S->st);
    if (S->prep) (void)hipStreamDestroy(S->prep);
    S->cv_done.notify_all();
    delete S;
    ctx->serve = nullptr;
    ctx->serving = false;
}

extern "C" gs_status gs_serve_start(gs_ctx *ctx, int32_t n_resident, const int32_t *designs, const int32_t *stims,
                                    const int32_t *resident_begin, const int32_t *resident_cycles, int32_t max_queue)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->serve) return gs_fail(ctx, GS_E_STATE, "already serving");
    if (n_resident < 0 || (n_resident > 0 && (!designs || !stims || !resident_begin || !resident_cycles)))
        return gs_fail(ctx, GS_E_INVALID, "bad resident arrays");
    if (max_queue <= 0) return gs_fail(ctx, GS_E_INVALID, "max_queue must be positive");
    for (int32_t i = 0; i < n_resident; i++) {
        Design *d = gs_get_design(ctx, designs[i]);
        if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", designs[i]);
        if (stims[i] < 0 || stims[i] >= (int32_t)ctx->stims.size() || ctx->stims[stims[i]]->design != designs[i])
            return gs_fail(ctx, GS_E_INVALID, "stimulus %d does not belong to design %d", stims[i], designs[i]);
        if (ctx->stims[stims[i]]->carry) return gs_fail(ctx, GS_E_INVALID, "continuous views are not served");
        if (resident_cycles[i] <= 0) return gs_fail(ctx, GS_E_INVALID, "resident window must be non-empty");
        gs_status st = gs_check_ranges(ctx, d, ctx->stims[stims[i]], resident_begin[i], resident_begin[i] + resident_cycles[i]);
        if (st) return st;
    }
    (void)hipSetDevice(ctx->opt.device);
    (void)hipStreamSynchronize(ctx->stream);
    gs_window_release(ctx, &ctx->win);          // the pool takes over the waveform budget
    gs_graph_cache_clear(ctx);
    ServeState *S = new ServeState();
    S->max_queue = max_queue;
    auto fail = [&](gs_status st, const char *msg) {
        ctx->serve = S;
        gs_serve_shutdown(ctx);
        return gs_fail(ctx, st, "%s", msg);
    };
    if (hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->prep, hipStreamNonBlocking) != hipSuccess)
        return fail(GS_E_DEVICE, "stream creation failed");
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    uint64_t pool_bytes = std::min<uint64_t>(ctx->budget, (uint64_t)(0.9 * (double)fr));
    pool_bytes &= ~255ull;
    if (hipMalloc(&S->pool_ptr, pool_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_E_NOMEM, "cannot allocate the serving pool");
    }
    S->pool.init((char *)S->pool_ptr, pool_bytes);
    S->seg_cap = 1024;
    if (hipMalloc((void **)&S->seg_ring, sizeof(Seg) * S->seg_cap * kRing) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_E_NOMEM, "cannot allocate segment tables");
    }
    for (int i = 0; i < kRing; i++)
        if (hipEventCreateWithFlags(&S->ring_ev[i], hipEventDisableTiming) != hipSuccess) return fail(GS_E_DEVICE, "event");
    if (hipHostMalloc((void **)&S->h_seg_ring, sizeof(Seg) * S->seg_cap * kRing, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&S->h_small, 4u << 20, hipHostMallocDefault) != hipSuccess)
        return fail(GS_E_NOMEM, "cannot allocate pinned staging buffers");
    int32_t max_n = 1;
    for (Design *d : ctx->designs)
        if (d) max_n = std::max(max_n, d->N);
    S->pinned_bytes = (uint64_t)kSaifArrays * 8 * max_n + 16 + 8ull * kMaxStripes * kBumpStride;
    for (int i = 0; i < kPinned; i++)
        if (hipHostMalloc(&S->pinned[i], S->pinned_bytes, hipHostMallocDefault) != hipSuccess)
            return fail(GS_E_NOMEM, "cannot allocate pinned result buffers");
    // resident windows: simulated once, kept in the pool
    std::string err;
    for (int32_t i = 0; i < n_resident; i++) {
        Req q;
        q.r.kind = GS_REQ_WINDOW;
        q.r.design = designs[i];
        q.r.stim = stims[i];
        q.r.cycle_begin = resident_begin[i];
        q.r.cycle_end = resident_begin[i] + resident_cycles[i];
        q.d = ctx->designs[designs[i]];
        q.s = ctx->stims[stims[i]];
        gs_status st = GS_OK;
        for (;;) {
            bool fits = true;
            st = admit(ctx, S, q, fits, err);
            if (st) break;
            if (!fits) { st = GS_E_NOMEM; err = "resident windows exceed the pool"; break; }
            st = start_request(ctx, S, q, err);
            if (st) break;
            std::vector<ReqP> one{std::shared_ptr<Req>(&q, [](Req *) {})};
            while (!st && q.next < q.lvl_n.size()) st = launch_step(ctx, S, one, err);
            if (st) break;
            unsigned int fl[4];
            if (hipMemcpyAsync(fl, q.flags, sizeof(fl), hipMemcpyDeviceToHost, S->st) != hipSuccess ||
                hipStreamSynchronize(S->st) != hipSuccess) { st = GS_E_DEVICE; err = "resident window"; break; }
            if (fl[3]) { st = GS_E_DEVICE; err = "internal error: an output chunk exceeded its fanin bound"; break; }
            if (fl[1]) { st = GS_E_CAPACITY; err = "resident window exceeds 32767 transitions per chunk"; break; }
            if (!fl[0]) break;
            S->pool.release(q.region);
            q.region = Region();
            q.arena_words *= 2;
        }
        if (st) return fail(st, err.c_str());
        Resident R;
        R.design = designs[i];
        R.stim = stims[i];
        R.c0 = q.c0;
        R.cycles = q.cycles;
        R.tiles = q.tiles;
        R.region = q.region;
        R.hdr = q.view.hdr;
        R.ends = q.view.ends;
        R.saif = q.acc.tc;
        S->res.push_back(R);
    }
    ctx->serve = S;
    ctx->serving = true;
    S->th = std::thread(serve_loop, ctx, S);
    return GS_OK;
}

extern "C" gs_status gs_submit(gs_ctx *ctx, const gs_request *req, uint64_t *ticket)
{
    ServeState *S = serve_of(ctx);
    if (!S) return gs_fail(ctx, GS_E_STATE, "not serving");
    if (!req || !ticket) return gs_fail(ctx, GS_E_INVALID, "null argument");
    auto q = std::make_shared<Req>();
    q->r = *req;
    q->t_submit = gs_now_ns();
    Design *d = gs_get_design(ctx, req->design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", req->design);
    if (req->stim < 0 || req->stim >= (int32_t)ctx->stims.size() || ctx->stims[req->stim]->design != req->design)
        return gs_fail(ctx, GS_E_INVALID, "stimulus %d does not belong to design %d", req->stim, req->design);
    if (ctx->stims[req->stim]->carry) return gs_fail(ctx, GS_E_INVALID, "continuous views are not served");
    q->d = d;
    q->s = ctx->stims[req->stim];
    if (req->kind == GS_REQ_WINDOW) {
        if (req->cycle_end <= req->cycle_begin) return gs_fail(ctx, GS_E_INVALID, "empty window");
        gs_status st = gs_check_ranges(ctx, d, q->s, req->cycle_begin, req->cycle_end);
        if (st) return st;
    } else if (req->kind == GS_REQ_EDIT) {
        if (req->n_edits <= 0 || !req->edits) return gs_fail(ctx, GS_E_INVALID, "an edit request needs edits");
        q->edits.assign(req->edits, req->edits + req->n_edits);
        q->r.edits = nullptr;
        for (size_t i = 0; i < S->res.size(); i++)
            if (S->res[i].design == req->design && S->res[i].stim == req->stim) q->res_idx = (int32_t)i;
        if (q->res_idx < 0) return gs_fail(ctx, GS_E_STATE, "no resident window for design %d, stimulus %d", req->design, req->stim);
    } else {
        return gs_fail(ctx, GS_E_INVALID, "unknown request kind");
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return gs_fail(ctx, S->fatal, "serving failed: %s", S->fatal_msg.c_str());
    if ((int32_t)S->queue.size() >= S->max_queue) return gs_fail(ctx, GS_E_BUSY, "admission queue is full");
    q->ticket = S->next_ticket++;
    S->queue.push_back(q);
    S->all[q->ticket] = q;
    *ticket = q->ticket;
    S->cv.notify_all();
    return GS_OK;
}

extern "C" gs_status gs_poll(gs_ctx *ctx, uint64_t ticket, int32_t wait, gs_result *res)
{
    ServeState *S = serve_of(ctx);
    if (!S) return gs_fail(ctx, GS_E_STATE, "not serving");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return gs_fail(ctx, GS_E_INVALID, "unknown ticket");
    ReqP q = it->second;
    if (wait) S->cv_done.wait(lk, [&] { return q->state == Q_DONE; });
    if (q->state != Q_DONE) return GS_E_BUSY;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->status = q->status;
        res->n_nets = q->d->N;
        res->tc = q->status == GS_OK ? q->tc.data() : nullptr;
        res->t0 = q->status == GS_OK ? q->t0.data() : nullptr;
        res->t1 = q->status == GS_OK ? q->t1.data() : nullptr;
        res->ig = q->status == GS_OK ? q->ig.data() : nullptr;
        res->gate_cycles = q->gate_cycles;
        res->t_submit_ns = q->t_submit;
        res->t_admit_ns = q->t_admit;
        res->t_done_ns = q->t_done;
    }
    if (q->status != GS_OK) ctx->err = q->err;
    return GS_OK;
}

extern "C" gs_status gs_release(gs_ctx *ctx, uint64_t ticket)
{
    ServeState *S = serve_of(ctx);
    if (!S) return gs_fail(ctx, GS_E_STATE, "not serving");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return gs_fail(ctx, GS_E_INVALID, "unknown ticket");
    if (it->second->state != Q_DONE) return gs_fail(ctx, GS_E_BUSY, "request still running");
    S->all.erase(it);
    return GS_OK;
}

extern "C" gs_status gs_serve_stop(gs_ctx *ctx)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (!ctx->serve) return gs_fail(ctx, GS_E_STATE, "not serving");
    gs_serve_shutdown(ctx);
    return GS_OK;
}
