// Level schedule: rounds of (design, stimulus, window) pieces evaluated
// level by level (GATSPI Section 3: a level starts once the previous level is
// complete), as direct launches or as one captured HIP graph per round shape;
// the plain simulate call, the batched call and the autotuner are built on it.
#include "host.h"

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

using namespace gs;

static_assert(kScratchBytes == GS_SCRATCH_BYTES, "the public scratch size and the device array differ");
static_assert(sizeof(Seg) == 176, "segment table capacity of the static scratch is documented for 176-byte segments");

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return gs_fail(ctx, GS_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

namespace {

struct Piece {
    Design *d;
    Stim *s;
    int32_t di, si;          // ids
    int32_t c0, cycles;
    uint64_t chunk_base;
    int32_t tiles;
};

struct Tuning {
    int32_t cap, wpb, tpw;
};

struct RoundResult {
    bool retry = false;
    double gate_eval_ms = 0, expand_ms = 0, round_ms = 0;
    int64_t launches = 0;
};

Tuning current_tuning(const gs_ctx *ctx)
{
    return Tuning{ctx->opt.lds_cap, ctx->opt.waves_per_block, ctx->opt.tiles_per_wave};
}

// The tuning for a round of pieces: the context's, except that an LDS
// output cap left to the library is sized by the densest piece's input
// toggles per (input, cycle).  A lane of a segment view carries the events
// of many cycles; with the single-cycle cap most of its lanes would take
// the spill path.
// Continuous views carry state from a wave's lane to the next, so each
// wave must start at a segment start: segments that tile 64 cycles allow
// any tiles per wave, others take whole windows (which start at segment
// starts) per wave.
Tuning carry_tuning(Tuning t, const std::vector<Piece> &ps)
{
    for (const Piece &p : ps)
        if (p.s->carry > 0 && kLanes % p.s->carry != 0) t.tpw = std::max(t.tpw, p.tiles);
    return t;
}

Tuning tuning_for(const gs_ctx *ctx, const std::vector<Piece> &ps)
{
    Tuning t = current_tuning(ctx);
    if (!ctx->auto_cap) return carry_tuning(t, ps);
    // inputs alone underrate designs whose logic multiplies glitches: take
    // the transitions per (net, cycle) seen when the design last ran too
    double rho = 0;
    for (const Piece &p : ps) {
        const int64_t tog = p.s->tog_prefix[p.c0 + p.cycles] - p.s->tog_prefix[p.c0];
        rho = std::max(rho, (double)tog / ((double)std::max(1, p.d->I) * std::max(1, p.cycles)));
        rho = std::max(rho, p.d->words_per_ps * (double)p.s->period);
    }
    t.cap = rho <= 0.5 ? 8 : rho <= 1.0 ? 16 : rho <= 3.0 ? 24 : 32;
    while (t.wpb > 1 && gate_eval_lds_bytes(t.cap, t.wpb) > ctx->lds_limit) t.wpb /= 2;   // fit the block's LDS
    return carry_tuning(t, ps);
}

uint64_t chunks_of(const Piece &p)
{
    return (uint64_t)p.d->N * (uint64_t)p.tiles;
}

// Release of dead nets: where each arena region of a round's pieces goes.
// Regions are numbered piece by piece, the design's regions in order.
struct RegionPlan {
    std::vector<size_t> piece_base;          // first region of each piece
    std::vector<uint64_t> off, slice;        // per region: first word, words per stripe
    std::vector<uint32_t> stripes;
    uint64_t peak = 0;                       // arena words the placement needs
    size_t counters = 0;                     // u64 stripe counters of all regions
};

constexpr uint32_t kRegionStripes = 16;

// Words to set aside for region r of a piece: the inputs' toggles exactly;
// for gate outputs the region's learned density (else the design's, else 2
// transitions per (net, cycle)) with 15% to spare, times the region's growth
// factor.  Stripes get 1,024 words more each for the uneven spread of
// reservations over them (plan_regions).
uint64_t region_words(const Piece &p, int32_t r)
{
    const Design *d = p.d;
    const int64_t nets = d->region_nets[r];
    if (nets == 0) return 0;
    double w;
    if (r == 0) {
        w = (double)(p.s->tog_prefix[p.c0 + p.cycles] - p.s->tog_prefix[p.c0]);
    } else {
        double wpp = d->region_wpp[r] > 0 ? d->region_wpp[r] : d->words_per_ps;
        if (wpp <= 0) wpp = 2.0 / (double)p.s->period;
        w = wpp * (double)nets * (double)p.cycles * (double)p.s->period;
    }
    return (uint64_t)(w * 1.15 * d->region_grow[r]) + 1;
}

gs_status region_alloc(gs_ctx *ctx, void **p, size_t bytes)
{
    if (ctx->noalloc || hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return gs_fail(ctx, GS_E_NOMEM, "cannot allocate the arena regions' table and counters");
    }
    return GS_OK;
}

// Places the regions first fit over the level steps: a region is taken
// before the first level that writes into it (the expansion, for the
// inputs) and given back once the last level that reads it has run.
void plan_regions(const std::vector<Piece> &ps, RegionPlan &pl)
{
    struct Item {
        int32_t first, last;
        size_t k;
    };
    pl = RegionPlan();
    std::vector<Item> items;
    for (const Piece &p : ps) {
        pl.piece_base.push_back(pl.off.size());
        for (int32_t r = 0; r < (int32_t)p.d->region_nets.size(); r++) {
            const uint64_t est = region_words(p, r);
            uint32_t stripes = 1;
            while (stripes < kRegionStripes && est / (2ull * stripes) >= 4096) stripes *= 2;
            const uint64_t slice = ((est + stripes - 1) / stripes + 1024 + 63) & ~63ull;
            pl.off.push_back(0);
            pl.slice.push_back(est ? slice : 0);
            pl.stripes.push_back(stripes);
            if (est) items.push_back({p.d->region_first[r], p.d->region_last[r], pl.off.size() - 1});
        }
    }
    pl.counters = pl.off.size() * kRegionStripes * kBumpStride;
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.first < b.first; });
    std::vector<std::pair<uint64_t, uint64_t>> gaps;        // free (first word, words), by address
    std::vector<Item> live;
    uint64_t top = 0;
    for (const Item &it : items) {
        for (size_t i = 0; i < live.size();) {
            if (live[i].last < it.first) {
                gaps.push_back({pl.off[live[i].k], pl.slice[live[i].k] * pl.stripes[live[i].k]});
                live[i] = live.back();
                live.pop_back();
            } else {
                i++;
            }
        }
        std::sort(gaps.begin(), gaps.end());
        std::vector<std::pair<uint64_t, uint64_t>> merged;
        for (const auto &g : gaps) {
            if (!merged.empty() && merged.back().first + merged.back().second == g.first) merged.back().second += g.second;
            else merged.push_back(g);
        }
        if (!merged.empty() && merged.back().first + merged.back().second == top) {
            top = merged.back().first;
            merged.pop_back();
        }
        gaps.swap(merged);
        const uint64_t n = pl.slice[it.k] * pl.stripes[it.k];
        size_t f = 0;
        while (f < gaps.size() && gaps[f].second < n) f++;
        if (f < gaps.size()) {
            pl.off[it.k] = gaps[f].first;
            gaps[f].first += n;
            gaps[f].second -= n;
            if (gaps[f].second == 0) gaps.erase(gaps.begin() + (long)f);
        } else {
            pl.off[it.k] = top;
            top += n;
        }
        pl.peak = std::max(pl.peak, top);
        live.push_back(it);
    }
}

// Builds the segment tables of every level step of a round: step l holds one
// segment per piece whose design has at least l levels.
void build_steps(gs_ctx *ctx, const std::vector<Piece> &pieces, const std::vector<WinView> &views, const Tuning &tu,
                 std::vector<Seg> &segs, std::vector<size_t> &step_off, std::vector<size_t> &step_n,
                 std::vector<uint64_t> &step_waves, std::vector<int32_t> &step_kmax, std::vector<int32_t> &step_wires)
{
    int32_t maxL = 0;
    for (const Piece &p : pieces) maxL = std::max(maxL, p.d->L);
    uint64_t salt = 0;
    for (const Piece &p : pieces) salt += ((uint64_t)p.d->I * p.tiles + 3) / 4;
    for (int32_t l = 1; l <= maxL; l++) {
        step_off.push_back(segs.size());
        uint64_t waves = 0;
        int32_t kmax = 1, wires = 0;
        for (size_t i = 0; i < pieces.size(); i++) {
            const Piece &p = pieces[i];
            if (p.d->L < l) continue;
            const uint32_t n_gates = p.d->level_ptr[l + 1] - p.d->level_ptr[l];
            if (n_gates == 0) continue;
            const uint64_t ngroup = ((uint64_t)p.tiles + tu.tpw - 1) / tu.tpw;
            Seg g;
            std::memset(&g, 0, sizeof(g));
            g.wave_begin = waves;
            g.gates = p.d->d_gates;
            g.pins = p.d->d_pins;
            g.gate_begin = p.d->level_ptr[l];
            g.n_gates = n_gates;
            g.salt = (uint32_t)salt;
            g.mode = (ctx->opt.wire_transport ? 1u : 0u) | ((uint32_t)std::max(0, p.s->carry) << 8);
            g.win = views[i];
            g.saif = saif_view(p.d->d_stage, (size_t)p.d->N);
            const uint64_t nw = (uint64_t)n_gates * ngroup;
            waves += nw;
            salt += (nw + tu.wpb - 1) / tu.wpb * tu.tpw;
            kmax = std::max(kmax, p.d->level_kmax[l]);
            wires |= p.d->has_wires ? 1 : 0;
            segs.push_back(g);
        }
        step_n.push_back(segs.size() - step_off.back());
        step_waves.push_back(waves);
        step_kmax.push_back(kmax);
        step_wires.push_back(wires);
    }
}

// Records the device work of one round on stream hs: clear flags and stripe
// counters, clear the SAIF staging of every design in the round, expand the
// stimulus of every piece, one gate-evaluation launch per level step, and
// (when commit) add the staging into the designs' SAIF accumulators unless a
// flag is set.  With timing, events bracket every launch (direct mode only).
gs_status record_round(gs_ctx *ctx, hipStream_t hs, const std::vector<Piece> &pieces, const std::vector<WinView> &views,
                       const std::vector<Design *> &designs, const Seg *d_segs, const std::vector<size_t> &step_off,
                       const std::vector<size_t> &step_n, const std::vector<uint64_t> &step_waves,
                       const std::vector<int32_t> &step_kmax, const std::vector<int32_t> &step_wires, const Tuning &tu,
                       bool commit, bool timing, uint64_t region_counters)
{
    size_t ev = 0;
    HIPCHK(launch_fill_u64(ctx->d_misc, 4, 0ull, hs));
    HIPCHK(launch_fill_u64(ctx->d_bump, (uint64_t)kMaxStripes * kBumpStride, 0ull, hs));
    if (region_counters) HIPCHK(launch_fill_u64(ctx->d_rbump, region_counters, 0ull, hs));
    for (Design *d : designs) HIPCHK(launch_fill_u64(d->d_stage, kSaifArrays * (uint64_t)d->N, 0ull, hs));
    if (timing) HIPCHK(hipEventRecord(gs_event(ctx, ev++), hs));
    for (size_t i = 0; i < pieces.size(); i++) {
        const Piece &p = pieces[i];
        StimView sv{p.s->d_init, p.s->d_tp, p.s->d_ts, p.d->I, p.s->period, p.s->carry};
        SaifAcc stage = saif_view(p.d->d_stage, (size_t)p.d->N);
        HIPCHK(launch_expand(sv, views[i], stage, ctx->d_c0 + i, (uint32_t)(i * 977), hs));
    }
    if (timing) HIPCHK(hipEventRecord(gs_event(ctx, ev++), hs));
    for (size_t k = 0; k < step_off.size(); k++) {
        if (step_waves[k] == 0) continue;
        if (timing) HIPCHK(hipEventRecord(gs_event(ctx, ev++), hs));
        HIPCHK(launch_gate_eval(d_segs + step_off[k], (int32_t)step_n[k], step_waves[k], step_wires[k], tu.cap, tu.wpb,
                                step_kmax[k], (uint32_t)tu.tpw, 0, pieces.front().s->carry > 0 ? 1 : 0, hs));
        if (timing) HIPCHK(hipEventRecord(gs_event(ctx, ev++), hs));
    }
    if (commit)
        for (Design *d : designs)
            HIPCHK(launch_add_u64_guarded(d->d_saif, d->d_stage, kSaifArrays * (uint64_t)d->N, (const unsigned int *)(ctx->d_misc + 1), hs));
    return GS_OK;
}

// Runs one round.  Window buffers must hold every piece's chunks and
// arena_words of transitions.
gs_status run_round(gs_ctx *ctx, std::vector<Piece> &pieces, uint64_t arena_words, const Tuning &tu, bool commit,
                    bool timing, RoundResult &res, const RegionPlan *plan = nullptr)
{
    hipStream_t hs = ctx->stream;
    res = RoundResult();
    uint64_t nch = 0;
    for (Piece &p : pieces) {
        p.chunk_base = nch;
        nch += chunks_of(p);
    }
    gs_status st = gs_window_reserve(ctx, &ctx->win, nch, arena_words);
    if (st) return st;
    std::vector<WinView> views;
    for (const Piece &p : pieces) views.push_back(gs_make_view(ctx, ctx->win, p.cycles, p.s->period, p.chunk_base, chunks_of(p)));
    if (plan) {
        // the region table and the regions' stripe counters
        const size_t nr = plan->off.size();
        if (ctx->regions_cap < nr) {
            gs_dev_free(ctx->d_regions);
            ctx->d_regions = nullptr;
            ctx->regions_cap = 0;
            void *p;
            if ((st = region_alloc(ctx, &p, sizeof(ArenaRegion) * nr))) return st;
            ctx->d_regions = (ArenaRegion *)p;
            ctx->regions_cap = nr;
        }
        if (ctx->rbump_cap < plan->counters) {
            gs_dev_free(ctx->d_rbump);
            ctx->d_rbump = nullptr;
            ctx->rbump_cap = 0;
            void *p;
            if ((st = region_alloc(ctx, &p, sizeof(unsigned long long) * plan->counters))) return st;
            ctx->d_rbump = (unsigned long long *)p;
            ctx->rbump_cap = plan->counters;
        }
        std::vector<ArenaRegion> tab(nr);
        for (size_t k = 0; k < nr; k++)
            tab[k] = ArenaRegion{plan->off[k], plan->slice[k], ctx->d_rbump + k * kRegionStripes * kBumpStride,
                                 plan->stripes[k] - 1, 0};
        HIPCHK(hipMemcpyAsync(ctx->d_regions, tab.data(), sizeof(ArenaRegion) * nr, hipMemcpyHostToDevice, hs));
        for (size_t i = 0; i < pieces.size(); i++) views[i].regions = ctx->d_regions + plan->piece_base[i];
    }
    std::vector<Design *> designs;
    for (const Piece &p : pieces)
        if (std::find(designs.begin(), designs.end(), p.d) == designs.end()) designs.push_back(p.d);
    std::vector<Seg> segs;
    std::vector<size_t> step_off, step_n;
    std::vector<uint64_t> step_waves;
    std::vector<int32_t> step_kmax, step_wires;
    build_steps(ctx, pieces, views, tu, segs, step_off, step_n, step_waves, step_kmax, step_wires);
    // per-piece first cycle lives in device memory so that a captured graph
    // can be replayed for another window of the same shape
    if (ctx->c0_cap < pieces.size()) {
        if (ctx->noalloc) return gs_fail(ctx, GS_E_NOMEM, "round parameter block outgrows the static scratch");
        gs_dev_free(ctx->d_c0);
        ctx->d_c0 = nullptr;
        ctx->c0_cap = 0;
        if (hipMalloc((void **)&ctx->d_c0, sizeof(int32_t) * std::max<size_t>(pieces.size(), 64)) != hipSuccess) {
            (void)hipGetLastError();
            return gs_fail(ctx, GS_E_NOMEM, "cannot allocate the round parameter block");
        }
        ctx->c0_cap = std::max<size_t>(pieces.size(), 64);
    }
    std::vector<int32_t> c0s;
    for (const Piece &p : pieces) c0s.push_back(p.c0);

    const bool graph = ctx->opt.schedule == GS_SCHED_GRAPH;
    const uint64_t t0 = gs_now_ns();
    if (!graph) {
        if ((st = gs_ensure_segs(ctx, std::max<size_t>(segs.size(), 1)))) return st;
        if (!segs.empty())
            HIPCHK(hipMemcpyAsync(ctx->d_segs, segs.data(), sizeof(Seg) * segs.size(), hipMemcpyHostToDevice, hs));
        HIPCHK(hipMemcpyAsync(ctx->d_c0, c0s.data(), sizeof(int32_t) * c0s.size(), hipMemcpyHostToDevice, hs));
        if ((st = record_round(ctx, hs, pieces, views, designs, ctx->d_segs, step_off, step_n, step_waves, step_kmax,
                               step_wires, tu, commit, timing, plan ? plan->counters : 0)))
            return st;
    } else {
        // graph key: everything the recorded launches depend on except the first cycles
        std::string key;
        auto add = [&key](uint64_t v) { key.append((const char *)&v, sizeof(v)); };
        add((uint64_t)(uintptr_t)ctx->win.hdr); add((uint64_t)(uintptr_t)ctx->win.ends);
        add((uint64_t)(uintptr_t)ctx->win.times); add(ctx->win.words); add((uint64_t)(uintptr_t)ctx->d_c0);
        add((uint64_t)tu.cap); add((uint64_t)tu.wpb); add((uint64_t)tu.tpw); add(commit);
        add(plan ? (uint64_t)(uintptr_t)ctx->d_regions : 0); add(plan ? (uint64_t)(uintptr_t)ctx->d_rbump : 0);
        add(plan ? (uint64_t)plan->counters : 0);
        for (const Piece &p : pieces) {
            add((uint64_t)p.di); add((uint64_t)p.si); add((uint64_t)p.cycles); add(p.d->version);
        }
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            if (ctx->graphs.size() >= 32) gs_graph_cache_clear(ctx);
            GraphEntry ge;
            if (hipMalloc((void **)&ge.segs, sizeof(Seg) * std::max<size_t>(segs.size(), 1)) != hipSuccess) {
                (void)hipGetLastError();
                return gs_fail(ctx, GS_E_NOMEM, "cannot allocate a graph's segment table");
            }
            if (!segs.empty())
                HIPCHK(hipMemcpyAsync(ge.segs, segs.data(), sizeof(Seg) * segs.size(), hipMemcpyHostToDevice, hs));
            HIPCHK(hipStreamSynchronize(hs));
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            gs_status rs = record_round(ctx, ctx->cap_stream, pieces, views, designs, ge.segs, step_off, step_n,
                                        step_waves, step_kmax, step_wires, tu, commit, false,
                                        plan ? plan->counters : 0);
            hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
            if (rs) {
                if (g) (void)hipGraphDestroy(g);
                gs_dev_free(ge.segs);
                return rs;
            }
            if (ce != hipSuccess) {
                gs_dev_free(ge.segs);
                return gs_fail(ctx, GS_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ce));
            }
            hipError_t ie = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                gs_dev_free(ge.segs);
                return gs_fail(ctx, GS_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ie));
            }
            it = ctx->graphs.emplace(key, ge).first;
        }
        HIPCHK(hipMemcpyAsync(ctx->d_c0, c0s.data(), sizeof(int32_t) * c0s.size(), hipMemcpyHostToDevice, hs));
        HIPCHK(hipEventRecord(gs_event(ctx, 0), hs));
        HIPCHK(hipStreamWaitEvent(ctx->cap_stream, ctx->events[0], 0));
        HIPCHK(hipGraphLaunch(it->second.exec, ctx->cap_stream));
        HIPCHK(hipEventRecord(gs_event(ctx, 1), ctx->cap_stream));
        HIPCHK(hipStreamWaitEvent(hs, ctx->events[1], 0));
        ctx->stats.graph_launches++;
    }
    unsigned long long hflags[4];
    std::vector<unsigned long long> hb((size_t)kMaxStripes * kBumpStride);
    HIPCHK(hipMemcpyAsync(hflags, ctx->d_misc, sizeof(hflags), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(hb.data(), ctx->d_bump, sizeof(unsigned long long) * hb.size(), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    res.round_ms = (gs_now_ns() - t0) * 1e-6;
    const unsigned int *f32 = (const unsigned int *)(hflags + 1);
    if (timing && !graph) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]));
        res.expand_ms += ms;
        size_t e = 2;
        for (size_t k = 0; k < step_off.size(); k++) {
            if (step_waves[k] == 0) continue;
            HIPCHK(hipEventElapsedTime(&ms, ctx->events[e], ctx->events[e + 1]));
            res.gate_eval_ms += ms;
            e += 2;
            res.launches++;
        }
    } else {
        for (size_t k = 0; k < step_off.size(); k++) res.launches += step_waves[k] ? 1 : 0;
    }
    const WinView &v0 = views.front();
    uint64_t used = 0;
    // words handed out: each stripe's counter less the words of its failed tries
    for (uint32_t i = 0; i <= v0.stripe_mask; i++)
        used += std::min<uint64_t>(hb[(size_t)i * kBumpStride] - hb[(size_t)i * kBumpStride + 1], v0.slice_words);
    std::vector<uint64_t> rused, rfailed;                   // per region (dead nets released)
    if (plan) {
        std::vector<unsigned long long> rb(plan->counters);
        HIPCHK(hipMemcpyAsync(rb.data(), ctx->d_rbump, sizeof(unsigned long long) * rb.size(), hipMemcpyDeviceToHost, hs));
        HIPCHK(hipStreamSynchronize(hs));
        const size_t nr = plan->off.size();
        rused.assign(nr, 0);
        rfailed.assign(nr, 0);
        for (size_t k = 0; k < nr; k++)
            for (uint32_t i = 0; i < plan->stripes[k]; i++) {
                const size_t c = (k * kRegionStripes + i) * kBumpStride;
                rused[k] += std::min<uint64_t>(rb[c] - rb[c + 1], plan->slice[k]);
                rfailed[k] += rb[c + 1];
            }
        used = 0;
        for (uint64_t u : rused) used += u;
        ctx->stats.release_peak_words = (int64_t)plan->peak;
        // a region that filled up gets twice the room in the next try
        for (size_t i = 0; i < pieces.size(); i++)
            for (size_t r = 0; r < pieces[i].d->region_nets.size(); r++)
                if (rfailed[plan->piece_base[i] + r]) pieces[i].d->region_grow[r] *= 2.0;
    }
    ctx->stats.arena_words = (int64_t)used;
    ctx->stats.spilled_lanes += f32[2];
    ctx->stats.unstaged_groups += f32[4];
    ctx->stats.queue_overflows += f32[5];
    if (f32[3]) return gs_fail(ctx, GS_E_DEVICE, "internal error: an output chunk exceeded its fanin bound");
    if (f32[1]) return gs_fail(ctx, GS_E_CAPACITY, "more than %u transitions in one (net, 64-cycle tile)", kMaxChunk);
    if (f32[0]) {
        res.retry = true;
        ctx->stats.window_retries++;
        return GS_OK;
    }
    if (commit && (ctx->d_profile || ctx->d_late))          // rounds that add nothing (pilots, trials) are not profiled
        for (const Piece &p : pieces) {
            const int64_t at = p.c0 - ctx->profile_begin;
            HIPCHK(launch_cycle_profile(ctx->win.ends + p.chunk_base * kLanes, ctx->win.hdr + p.chunk_base,
                                        ctx->win.times, ctx->d_wout, (uint32_t)p.d->N, (uint32_t)p.tiles,
                                        (uint32_t)p.cycles, p.s->period, ctx->d_profile ? ctx->d_profile + at : nullptr,
                                        ctx->d_late ? ctx->d_late + at : nullptr, hs));
        }
    // learn the design's list density from rounds of one design
    double lane_ps = 0;
    for (const Piece &p : pieces) lane_ps += (double)p.cycles * (double)p.s->period;
    if (designs.size() == 1 && lane_ps > 0) {
        Design *d = designs[0];
        d->words_per_ps = (double)used / ((double)std::max(1, d->N) * lane_ps);
        if (plan)                                           // and each region's
            for (size_t r = 1; r < d->region_nets.size(); r++) {
                if (!d->region_nets[r]) continue;
                uint64_t u = 0;
                for (size_t i = 0; i < pieces.size(); i++) u += rused[plan->piece_base[i] + r];
                d->region_wpp[r] = (double)u / ((double)d->region_nets[r] * lane_ps);
                d->region_grow[r] = 1.0;                    // the measured density replaces an earlier growth
            }
    }
    ctx->stats.gate_eval_ms += res.gate_eval_ms;
    ctx->stats.expand_ms += res.expand_ms;
    ctx->stats.gate_eval_launches += res.launches;
    ctx->stats.windows += (int64_t)pieces.size();
    for (const Piece &p : pieces) ctx->stats.gate_cycles += (int64_t)p.d->G * p.cycles;
    // the round's windows stay readable through gs_read_waveform (not when
    // the space of dead nets was reused)
    ctx->last.clear();
    ctx->last_released = plan != nullptr;
    for (const Piece &p : pieces) {
        if (plan) break;
        LastWindow lw;
        lw.design = p.di;
        lw.stim = p.si;
        lw.c0 = p.c0;
        lw.cycles = p.cycles;
        lw.chunk_base = p.chunk_base;
        lw.n_nets = p.d->N;
        ctx->last.push_back(lw);
    }
    return GS_OK;
}

uint64_t piece_arena_guess(const Piece &p)
{
    uint64_t g = gs_arena_guess(p.d->N, p.cycles, p.s->tog_prefix[p.c0 + p.cycles] - p.s->tog_prefix[p.c0]);
    // a design that ran before: its observed density with 15% to spare
    if (p.d->words_per_ps > 0)
        g = std::max<uint64_t>(g, (uint64_t)(p.d->words_per_ps * (double)p.s->period * 1.15 * (double)p.d->N *
                                             p.cycles) + (1ull << 20));
    return g;
}

// The first part of a window that has to be split, or 0 when it cannot be:
// halves, at least 64 cycles, and for a continuous view whole segments.
int32_t split_cycles(const Piece &p)
{
    const int32_t S = std::max(1, p.s->carry);
    if (p.cycles <= std::max(kLanes, S)) return 0;
    const int32_t a = p.cycles / 2 / S * S;
    return a > 0 ? a : S;
}

// Runs `pieces` as rounds that fit the budget.  A round whose arena fills up
// is retried with twice the arena; at the budget limit the round is split
// and, for a single piece, its window is halved.
gs_status run_pieces(gs_ctx *ctx, std::vector<Piece> pending, const Tuning &tu, bool commit, bool timing,
                     double *gate_eval_ms, uint64_t min_words = 0)
{
    std::reverse(pending.begin(), pending.end());      // pop from the back in submission order
    uint64_t grown = 0;
    size_t max_round = (size_t)-1;
    while (!pending.empty()) {
        // pack pieces while headers + arena guesses fit the budget
        std::vector<Piece> round;
        uint64_t hdr = 0, guess = 0;
        while (!pending.empty() && round.size() < max_round) {
            const Piece &p = pending.back();
            // a round's launches run either continuous views or none
            if (!round.empty() && (p.s->carry > 0) != (round.front().s->carry > 0)) break;
            const uint64_t hb = gs_header_bytes(p.d->N, p.cycles);
            const uint64_t gw = piece_arena_guess(p);
            if (!round.empty() && hdr + hb + (guess + gw) * sizeof(int32_t) > ctx->budget) break;
            round.push_back(p);
            pending.pop_back();
            hdr += hb;
            guess += gw;
        }
        if (hdr >= ctx->budget) {
            Piece p = round.front();
            if (round.size() == 1 && split_cycles(p) > 0) {     // halve the window
                Piece a = p, b = p;
                a.cycles = split_cycles(p);
                a.tiles = (a.cycles + kLanes - 1) / kLanes;
                b.c0 = p.c0 + a.cycles;
                b.cycles = p.cycles - a.cycles;
                b.tiles = (b.cycles + kLanes - 1) / kLanes;
                pending.push_back(b);
                pending.push_back(a);
                continue;
            }
            return gs_fail(ctx, GS_E_NOMEM, "budget cannot hold the chunk headers of one window");
        }
        const uint64_t max_words = (ctx->budget - hdr) / sizeof(int32_t);
        uint64_t words = std::min(max_words, std::max(std::max(guess, min_words), std::max(grown, ctx->win.words)));
        // dead nets released: the arena is what the regions' placement needs
        RegionPlan plan;
        if (ctx->releasing) {
            plan_regions(round, plan);
            if (plan.peak > max_words) {
                if (round.size() > 1) {
                    max_round = round.size() / 2;
                    for (auto it = round.rbegin(); it != round.rend(); ++it) pending.push_back(*it);
                    continue;
                }
                const int32_t a_cycles = split_cycles(round[0]);
                if (a_cycles <= 0)
                    return gs_fail(ctx, GS_E_NOMEM, "the arena regions of one %d-cycle window exceed the memory budget",
                                   round[0].cycles);
                Piece p = round[0], a = p, b = p;
                a.cycles = a_cycles;
                a.tiles = (a.cycles + kLanes - 1) / kLanes;
                b.c0 = p.c0 + a.cycles;
                b.cycles = p.cycles - a.cycles;
                b.tiles = (b.cycles + kLanes - 1) / kLanes;
                pending.push_back(b);
                pending.push_back(a);
                continue;
            }
            words = std::max<uint64_t>(plan.peak, std::min(max_words, ctx->win.words));
        }
        RoundResult rr;
        gs_status st = run_round(ctx, round, words, tu, commit, timing, rr, ctx->releasing ? &plan : nullptr);
        if (st) return st;
        if (gate_eval_ms) *gate_eval_ms += rr.gate_eval_ms;
        if (!rr.retry) continue;
        if (ctx->releasing) {
            // the regions that filled up were given twice the room: plan again
            for (auto it = round.rbegin(); it != round.rend(); ++it) pending.push_back(*it);
            continue;
        }
        // arena full: grow, else split the round, else halve the single window
        if (words < max_words) {
            grown = std::min(max_words, words * 2);
            for (auto it = round.rbegin(); it != round.rend(); ++it) pending.push_back(*it);
        } else if (round.size() > 1) {
            // fewer pieces per round: each round gets the whole arena
            max_round = round.size() / 2;
            for (auto it = round.rbegin(); it != round.rend(); ++it) pending.push_back(*it);
        } else if (split_cycles(round[0]) > 0) {
            Piece p = round[0], a = p, b = p;
            a.cycles = split_cycles(p);
            a.tiles = (a.cycles + kLanes - 1) / kLanes;
            b.c0 = p.c0 + a.cycles;
            b.cycles = p.cycles - a.cycles;
            b.tiles = (b.cycles + kLanes - 1) / kLanes;
            pending.push_back(b);
            pending.push_back(a);
        } else {
            return gs_fail(ctx, GS_E_NOMEM, "transitions of one %d-cycle window exceed the memory budget", round[0].cycles);
        }
    }
    return GS_OK;
}

Piece make_piece(gs_ctx *ctx, int32_t di, int32_t si, int32_t c0, int32_t cycles)
{
    Piece p;
    p.d = ctx->designs[di];
    p.s = ctx->stims[si];
    p.di = di;
    p.si = si;
    p.c0 = c0;
    p.cycles = cycles;
    p.chunk_base = 0;
    p.tiles = (cycles + kLanes - 1) / kLanes;
    return p;
}

// Window length for a design and a stimulus period: the caller's, else the
// longest power-of-two number of cycles up to 16,384 whose chunk headers
// take at most a third of the budget and, once the design's transition
// density is known, whose headers and transitions (with 15% to spare) fit
// the budget.
int32_t window_cycles(gs_ctx *ctx, const Design *d, int32_t period)
{
    int32_t W = ctx->opt.window_cycles;
    if (W <= 0) {
        W = 16384;
        while (W > kLanes && gs_header_bytes(d->N, W) * 3 > ctx->budget) W /= 2;
        if (d->words_per_ps > 0) {
            auto need = [&](int32_t w) {
                return (double)gs_header_bytes(d->N, w) +
                       d->words_per_ps * (double)period * 1.15 * (double)d->N * (double)w * sizeof(int32_t);
            };
            while (W > kLanes && need(W) > (double)ctx->budget) W /= 2;
        }
    }
    return W;
}

// The same for a stimulus.  A continuous view's windows hold whole
// segments.  Where segments do not tile 64 cycles, a wave takes a whole
// window, so windows are kept near 1,024 cycles (or one segment) and run
// several to a round, which keeps launches wide.
int32_t default_window(gs_ctx *ctx, const Design *d, const Stim *s)
{
    const int32_t W = window_cycles(ctx, d, s->period), S = s->carry;
    if (S <= 0) return W;
    if (kLanes % S != 0) return std::min(std::max(1, W / S), std::max(1, 1024 / S)) * S;
    return std::max(1, W / S) * S;
}

gs_status check_job(gs_ctx *ctx, int32_t design, int32_t stim, int32_t b, int32_t e)
{
    Design *d = gs_get_design(ctx, design);
    if (!d) return gs_fail(ctx, GS_E_INVALID, "no design %d", design);
    if (stim < 0 || stim >= (int32_t)ctx->stims.size() || !ctx->stims[stim] || ctx->stims[stim]->design != design)
        return gs_fail(ctx, GS_E_INVALID, "stimulus %d does not belong to design %d", stim, design);
    return gs_check_ranges(ctx, d, ctx->stims[stim], b, e);
}

}  // namespace

void gs_graph_cache_clear(gs_ctx *ctx)
{
    for (auto &kv : ctx->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        gs_dev_free(kv.second.segs);
    }
    ctx->graphs.clear();
}

extern "C" gs_status gs_cycle_profile(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end,
                                     int64_t *glitch, int64_t *late)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->serving) return gs_fail(ctx, GS_E_STATE, "context is serving; use gs_submit");
    gs_status st = check_job(ctx, design, stim, cycle_begin, cycle_end);
    if (st) return st;
    if (ctx->stims[stim]->carry) return gs_fail(ctx, GS_E_INVALID, "no cycle profile of a continuous view");
    if (ctx->opt.release_dead) return gs_fail(ctx, GS_E_INVALID, "no cycle profile when dead nets are released");
    const int32_t n = cycle_end - cycle_begin;
    (void)hipSetDevice(ctx->opt.device);
    const Design *d = ctx->designs[design];
    // per net: the slowest fanout wire for a rising and for a falling edge
    std::vector<int32_t> wout;
    if (late && d->has_wires) {
        wout.assign(2 * (size_t)d->N, 0);
        for (int64_t s = 0; s < d->F; s++) {
            const size_t net = (size_t)d->fanin_net[s];
            wout[2 * net] = std::max(wout[2 * net], d->wr[s]);
            wout[2 * net + 1] = std::max(wout[2 * net + 1], d->wf[s]);
        }
    }
    const size_t m = (size_t)std::max(n, 1);
    unsigned long long *buf = nullptr;
    int32_t *dw = nullptr;
    if (hipMalloc((void **)&buf, sizeof(unsigned long long) * 2 * m) != hipSuccess ||
        (!wout.empty() && hipMalloc((void **)&dw, sizeof(int32_t) * wout.size()) != hipSuccess)) {
        (void)hipGetLastError();
        gs_dev_free(buf);
        return gs_fail(ctx, GS_E_NOMEM, "cannot allocate the cycle profile");
    }
    hipError_t he = launch_fill_u64(buf, 2 * m, 0ull, ctx->stream);
    if (he == hipSuccess && dw)
        he = hipMemcpyAsync(dw, wout.data(), sizeof(int32_t) * wout.size(), hipMemcpyHostToDevice, ctx->stream);
    if (he != hipSuccess) {
        gs_dev_free(buf);
        gs_dev_free(dw);
        return gs_fail(ctx, GS_E_DEVICE, "%s", hipGetErrorString(he));
    }
    ctx->d_profile = glitch ? buf : nullptr;
    ctx->d_late = late ? buf + m : nullptr;
    ctx->d_wout = dw;
    ctx->profile_begin = cycle_begin;
    st = gs_simulate(ctx, design, stim, cycle_begin, cycle_end);
    ctx->d_profile = nullptr;
    ctx->d_late = nullptr;
    ctx->d_wout = nullptr;
    std::vector<unsigned long long> h(2 * m);
    if (!st && (hipMemcpyAsync(h.data(), buf, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                               ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess))
        st = gs_fail(ctx, GS_E_DEVICE, "cycle profile readback failed");
    gs_dev_free(buf);
    gs_dev_free(dw);
    if (st) return st;
    for (int32_t c = 0; c < n; c++) {
        if (glitch) glitch[c] = (int64_t)h[c];
        if (late) late[c] = (int64_t)h[m + c];
    }
    return GS_OK;
}

extern "C" gs_status gs_glitch_profile(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin,
                                      int32_t cycle_end, int64_t *per_cycle)
{
    if (ctx && cycle_end > cycle_begin && !per_cycle) return gs_fail(ctx, GS_E_INVALID, "null per_cycle");
    return gs_cycle_profile(ctx, design, stim, cycle_begin, cycle_end, per_cycle, nullptr);
}

extern "C" gs_status gs_simulate(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->serving) return gs_fail(ctx, GS_E_STATE, "context is serving; use gs_submit");
    gs_status st = gs_job_cycles(ctx, stim, cycle_begin, cycle_end);
    if (st) return st;
    st = check_job(ctx, design, stim, cycle_begin, cycle_end);
    if (st) return st;
    (void)hipSetDevice(ctx->opt.device);
    const uint64_t t_start = gs_now_ns();
    ctx->last.clear();
    ctx->last_released = false;
    Design *d = ctx->designs[design];
    // release of dead nets applies to this call only (batches, the
    // allocation-free call and serving keep every net)
    struct Releasing {
        gs_ctx *c;
        ~Releasing() { c->releasing = false; }
    } releasing_guard{ctx};
    ctx->releasing = ctx->opt.release_dead != 0;
    // a design's first run learns its transition density from a 64-cycle
    // pilot (nothing committed), so that the arena of the real windows is
    // sized from it rather than guessed and retried
    if (d->words_per_ps <= 0 && cycle_end - cycle_begin > 2 * kLanes) {
        const Piece pilot = make_piece(ctx, design, stim, cycle_begin, kLanes);
        // room for 8 transitions per (net, cycle), so that the pilot itself
        // rarely needs a second try
        st = run_pieces(ctx, std::vector<Piece>{pilot}, tuning_for(ctx, {pilot}), false, false, nullptr,
                        8ull * (uint64_t)d->N * kLanes);
        if (st) return st;
    }
    const Stim *sm = ctx->stims[stim];
    const int32_t W = default_window(ctx, d, sm);
    std::vector<Piece> pieces;
    for (int32_t c0 = cycle_begin; c0 < cycle_end; c0 += W)
        pieces.push_back(make_piece(ctx, design, stim, c0, std::min(W, cycle_end - c0)));
    // windows are independent: as many to a round (one launch per level
    // for all of them) as the budget holds
    st = run_pieces(ctx, pieces, tuning_for(ctx, pieces), true, ctx->opt.timing != 0, nullptr);
    if (st) return st;
    ctx->stats.wall_ms += (gs_now_ns() - t_start) * 1e-6;
    return GS_OK;
}

// The allocation-free variant of gs_simulate.  Every buffer a round needs
// beyond the loaded design and stimulus comes from this GPU's static scratch,
// in this order: flags and counters, stripe counters, the first-cycle block,
// the segment table, then the window (chunk headers, lane ends, transition
// arena, carved as for a caller-owned arena).  Windows are as long as the
// headers fit in half of the window region; a full arena halves them.  The
// context's own buffers and options are restored on return.  Calls that
// overlap on one GPU share the scratch and race.
extern "C" gs_status gs_simulate_noalloc(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin,
                                         int32_t cycle_end)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->serving) return gs_fail(ctx, GS_E_STATE, "context is serving; use gs_submit");
    gs_status st = gs_job_cycles(ctx, stim, cycle_begin, cycle_end);
    if (st) return st;
    st = check_job(ctx, design, stim, cycle_begin, cycle_end);
    if (st) return st;
    if (!ctx->d_scratch) return gs_fail(ctx, GS_E_STATE, "no static scratch on this device");
    (void)hipSetDevice(ctx->opt.device);
    Design *d = ctx->designs[design];
    constexpr size_t kMiscBytes = 256, kBumpBytes = sizeof(unsigned long long) * kMaxStripes * kBumpStride;
    constexpr size_t kC0Slots = 64, kSegBytes = 1u << 20;
    char *base = ctx->d_scratch;
    char *misc = base, *bump = misc + kMiscBytes, *c0 = bump + kBumpBytes, *segs = c0 + 256;
    char *win = segs + kSegBytes;
    const size_t win_bytes = kScratchBytes - (size_t)(win - base);
    const size_t seg_cap = kSegBytes / sizeof(Seg);
    if ((size_t)d->L > seg_cap)
        return gs_fail(ctx, GS_E_NOMEM, "%d levels exceed the %zu segments of the static scratch", d->L, seg_cap);
    if (gs_header_bytes((uint64_t)d->N, kLanes) * 2 > win_bytes)
        return gs_fail(ctx, GS_E_NOMEM, "a 64-cycle window of %d nets needs %llu bytes of chunk headers and lane "
                       "ends; the static scratch holds %zu bytes for windows", d->N,
                       (unsigned long long)gs_header_bytes((uint64_t)d->N, kLanes), win_bytes);
    int32_t W = 16384;
    while (W > kLanes && gs_header_bytes((uint64_t)d->N, W) * 2 > win_bytes) W /= 2;
    const int32_t S = ctx->stims[stim]->carry;
    if (S > 0) {                                            // whole segments per window
        W = std::max(1, W / S) * S;
        if (gs_header_bytes((uint64_t)d->N, W) * 2 > win_bytes)
            return gs_fail(ctx, GS_E_NOMEM, "the chunk headers of one %d-cycle segment outgrow the static scratch", S);
    }

    struct Saved {
        gs_options opt;
        uint64_t budget;
        WindowBufs win;
        unsigned long long *misc, *bump;
        Seg *segs;
        size_t segs_cap;
        int32_t *c0;
        size_t c0_cap;
    } sv{ctx->opt, ctx->budget, ctx->win, ctx->d_misc, ctx->d_bump, ctx->d_segs, ctx->segs_cap, ctx->d_c0,
         ctx->c0_cap};
    ctx->opt.arena = win;
    ctx->opt.arena_bytes = win_bytes;
    ctx->opt.schedule = GS_SCHED_LEVELS;
    ctx->budget = win_bytes;
    ctx->win = WindowBufs();
    ctx->d_misc = (unsigned long long *)misc;
    ctx->d_bump = (unsigned long long *)bump;
    ctx->d_segs = (Seg *)segs;
    ctx->segs_cap = seg_cap;
    ctx->d_c0 = (int32_t *)c0;
    ctx->c0_cap = kC0Slots;
    ctx->noalloc = true;
    const uint64_t t_start = gs_now_ns();
    for (int32_t b = cycle_begin; b < cycle_end && st == GS_OK; b += W) {
        const Piece p = make_piece(ctx, design, stim, b, std::min(W, cycle_end - b));
        st = run_pieces(ctx, std::vector<Piece>{p}, tuning_for(ctx, {p}), true, false, nullptr);
    }
    if (st == GS_OK && hipStreamSynchronize(ctx->stream) != hipSuccess)
        st = gs_fail(ctx, GS_E_DEVICE, "stream synchronisation failed");
    ctx->noalloc = false;
    ctx->opt = sv.opt;
    ctx->budget = sv.budget;
    ctx->win = sv.win;
    ctx->d_misc = sv.misc;
    ctx->d_bump = sv.bump;
    ctx->d_segs = sv.segs;
    ctx->segs_cap = sv.segs_cap;
    ctx->d_c0 = sv.c0;
    ctx->c0_cap = sv.c0_cap;
    ctx->last.clear();                  // the scratch window is not kept for gs_read_waveform
    ctx->stats.wall_ms += (gs_now_ns() - t_start) * 1e-6;
    return st;
}

// Times each candidate tuning on a trial window (nothing committed) and
// keeps the fastest in the context.  The staging caps tried are the one
// the trial's toggle density calls for (or the caller's), half and twice it.
static gs_status autotune_impl(gs_ctx *ctx, const std::vector<Piece> &trial, Tuning *best_out, double *best_ms)
{
    const int32_t c = tuning_for(ctx, trial).cap;
    const int32_t lo = std::max(4, c / 2), hi = std::min(32, c * 2);
    const Tuning cands[] = {{c, 4, 8}, {c, 4, 4}, {c, 2, 8}, {c, 4, 16}, {hi, 4, 8}, {c, 8, 8}, {c, 4, 2}, {lo, 4, 8}};
    double best = 1e30;
    Tuning bt = current_tuning(ctx);
    const int saved_sched = ctx->opt.schedule;
    ctx->opt.schedule = GS_SCHED_LEVELS;              // events bracket every launch
    gs_stats saved = ctx->stats;
    for (const Tuning &t : cands) {
        if (gate_eval_lds_bytes(t.cap, t.wpb) > ctx->lds_limit) continue;     // does not fit the device
        double ms = 0;
        gs_status st = run_pieces(ctx, trial, t, false, true, &ms);   // warm
        if (st) { ctx->opt.schedule = saved_sched; ctx->stats = saved; return st; }
        ms = 0;
        st = run_pieces(ctx, trial, t, false, true, &ms);
        if (st) { ctx->opt.schedule = saved_sched; ctx->stats = saved; return st; }
        // the first candidate is the default shape; another replaces the
        // best so far only when it is clearly faster on the trial, which
        // stands in for the whole batch only approximately
        if (ms < (&t == cands ? best : 0.97 * best)) {
            best = ms;
            bt = t;
        }
    }
    ctx->opt.schedule = saved_sched;
    ctx->stats = saved;
    ctx->opt.lds_cap = bt.cap;
    ctx->opt.waves_per_block = bt.wpb;
    ctx->opt.tiles_per_wave = bt.tpw;
    ctx->auto_cap = false;                            // the tuned cap stays
    if (best_out) *best_out = bt;
    if (best_ms) *best_ms = best;
    return GS_OK;
}

extern "C" gs_status gs_autotune(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end,
                                 gs_tuning *out)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->serving) return gs_fail(ctx, GS_E_STATE, "context is serving");
    gs_status st = check_job(ctx, design, stim, cycle_begin, cycle_end);
    if (st) return st;
    if (ctx->stims[stim]->carry) return gs_fail(ctx, GS_E_INVALID, "tune on the stimulus, not its continuous view");
    if (cycle_end <= cycle_begin) return gs_fail(ctx, GS_E_INVALID, "empty trial range");
    (void)hipSetDevice(ctx->opt.device);
    std::vector<Piece> trial{make_piece(ctx, design, stim, cycle_begin, std::min(cycle_end - cycle_begin, 4096))};
    Tuning t;
    double ms;
    st = autotune_impl(ctx, trial, &t, &ms);
    if (st) return st;
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->lds_cap = t.cap;
        out->waves_per_block = t.wpb;
        out->tiles_per_wave = t.tpw;
        out->trial_ms = ms;
    }
    return GS_OK;
}

extern "C" gs_status gs_simulate_batch(gs_ctx *ctx, int32_t n_jobs, const gs_job *jobs)
{
    if (!ctx) return gs_fail(nullptr, GS_E_INVALID, "null context");
    if (ctx->serving) return gs_fail(ctx, GS_E_STATE, "context is serving; use gs_submit");
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return gs_fail(ctx, GS_E_INVALID, "bad job array");
    // jobs on continuous views count segments: as cycle ranges from here on
    std::vector<gs_job> cj(jobs, jobs + n_jobs);
    for (int32_t i = 0; i < n_jobs; i++) {
        gs_status st = gs_job_cycles(ctx, cj[i].stim, cj[i].cycle_begin, cj[i].cycle_end);
        if (st) return st;
        st = check_job(ctx, cj[i].design, cj[i].stim, cj[i].cycle_begin, cj[i].cycle_end);
        if (st) return st;
    }
    jobs = cj.data();
    (void)hipSetDevice(ctx->opt.device);
    const uint64_t t_start = gs_now_ns();
    ctx->last.clear();
    std::vector<Piece> pieces;
    for (int32_t i = 0; i < n_jobs; i++) {
        const gs_job &j = jobs[i];
        Design *d = ctx->designs[j.design];
        const int32_t W = default_window(ctx, d, ctx->stims[j.stim]);
        for (int32_t c0 = j.cycle_begin; c0 < j.cycle_end; c0 += W)
            pieces.push_back(make_piece(ctx, j.design, j.stim, c0, std::min(W, j.cycle_end - c0)));
    }
    if (pieces.empty()) return GS_OK;
    if (ctx->opt.autotune) {
        // tune once per batch shape on the batch itself, each piece cut to
        // at most 2,048 cycles: a trial of one piece, or of a few hundred
        // cycles, favours settings that lose on the whole uneven mix
        std::string key;
        for (const Piece &p : pieces) {
            key += std::to_string(p.di) + ":" + std::to_string(p.cycles) + ",";
        }
        auto it = ctx->tuned.find(key);
        if (it == ctx->tuned.end()) {
            std::vector<Piece> trial = pieces;
            for (Piece &p : trial) {
                p.cycles = std::min(p.cycles, 2048);
                p.tiles = (p.cycles + kLanes - 1) / kLanes;
            }
            Tuning t;
            double ms;
            gs_status st = autotune_impl(ctx, trial, &t, &ms);
            if (st) return st;
            ctx->tuned[key] = {t.cap, t.wpb, t.tpw};
        } else {
            ctx->opt.lds_cap = it->second[0];
            ctx->opt.waves_per_block = it->second[1];
            ctx->opt.tiles_per_wave = it->second[2];
        }
    }
    gs_status st = run_pieces(ctx, pieces, tuning_for(ctx, pieces), true, ctx->opt.timing != 0, nullptr);
    if (st) return st;
    ctx->stats.wall_ms += (gs_now_ns() - t_start) * 1e-6;
    return GS_OK;
}
