// Host-side structures of a context (not part of the public ABI).
#pragma once

#include "gatesim.h"
#include "internal.h"

#include <array>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

// Arc records of one fanin slot sorted by kind: kind = 3 * c + e with c = 0
// for an unconditional record, else 1 + its condition value, and e its
// input-edge qualifier (0 either edge, 1 rising, 2 falling).  Each entry is
// the record's index, -1 for none or -2 for more than one.
constexpr int kArcKinds = 9;

template <class R> inline int arc_kind(const R &a)
{
    return 3 * (a.cond_pin < 0 ? 0 : 1 + (a.cond_val ? 1 : 0)) + a.in_edge;
}

// The record that sets a slot's delays where its condition pin has value cv
// and its input edge is ie (1 rising): the most specific kind that applies
// (condition and edge; then condition alone or edge alone, which must not
// both exist; then neither).  -1: no record applies; -2: not unique.
inline int64_t arc_winner(const int64_t *kind, int cv, int ie)
{
    const int e = ie ? 1 : 2;
    const int64_t both = kind[3 * (1 + cv) + e];
    if (both != -1) return both;
    const int64_t c = kind[3 * (1 + cv)], x = kind[e];
    if (c != -1 && x != -1) return -2;
    if (c != -1) return c;
    if (x != -1) return x;
    return kind[0];
}

struct Design {
    int32_t I = 0, G = 0, N = 0, L = 0;
    int64_t F = 0;
    int32_t max_pins = 0;
    std::vector<uint8_t> gate_k;
    std::vector<uint64_t> gate_truth;
    std::vector<int64_t> fanin_ptr;
    std::vector<int32_t> fanin_net;
    std::vector<int32_t> level;          // per gate
    std::vector<int32_t> perm;           // level order -> gate
    std::vector<uint32_t> level_ptr;     // level l's gates: [level_ptr[l], level_ptr[l+1]), l = 1..L
    std::vector<int32_t> level_kmax;     // largest pin count in each level
    int32_t level_sweeps = 0;
    // compiled delays per fanin slot
    std::vector<int32_t> q, dl, wr, wf;  // dl: 8 per slot, PinRec::d order
    std::vector<int64_t> slot_rec;       // kArcKinds per slot, as arc_winner reads them
    std::vector<gs_arc> arcs;            // the loaded arc records
    bool arcs_loaded = false, has_wires = false;
    int32_t zero_delay = 0, max_delay = 0, max_wire = 0;
    uint64_t version = 0;
    // learned from earlier rounds, used for performance only: transition
    // words per net and picosecond of lane time in the last round that ran
    // this design alone (a segment view's lanes are longer); the window
    // planner and the arena guess size windows from it
    double words_per_ps = 0;
    // release of dead nets: arena regions (0: the inputs; then one per level
    // and class of last reading level, GateRec::dead); per region its net
    // count, the level that writes it, the last level that reads one of its
    // nets, and, learned, its transition words per net and picosecond and a
    // growth factor raised each time it filled up
    std::vector<int64_t> region_nets;
    std::vector<int32_t> region_first, region_last;
    std::vector<double> region_wpp, region_grow;
    // device
    int64_t *d_fanin_ptr = nullptr;
    int32_t *d_fanin_net = nullptr;
    int32_t *d_level = nullptr;
    gs::GateRec *d_gates = nullptr;
    gs::PinRec *d_pins = nullptr;
    unsigned long long *d_saif = nullptr;    // tc[N], t0[N], t1[N], ig[N] (SaifAcc order)
    unsigned long long *d_stage = nullptr;   // per-window staging, same layout
};

struct Stim {
    int32_t design = -1, period = 0, n_cycles = 0;
    int64_t n_toggles = 0;
    bool owns = true;                        // false: a segment view sharing another stimulus's arrays
    // > 0: a continuous view whose segments of `carry` cycles run one lane
    // per cycle, with the edge pending at each cycle's end carried into the
    // next; period and n_cycles stay those of single cycles, and the cycle
    // indices of calls that take the view count segments
    int32_t carry = 0;
    uint8_t *d_init = nullptr;
    int64_t *d_tp = nullptr;
    int64_t *d_ts = nullptr;
    std::vector<int64_t> tog_prefix;         // input toggles before cycle c
};

struct WindowBufs {
    gs::ChunkHdr *hdr = nullptr;
    uint16_t *ends = nullptr;
    int32_t *times = nullptr;
    uint64_t chunks = 0;                     // capacity in (net, tile) chunks
    uint64_t words = 0;                      // capacity of `times`
};

struct LastWindow {
    int32_t design = -1, stim = -1, c0 = 0, cycles = 0;
    uint64_t chunk_base = 0;
    int32_t n_nets = 0;
};

struct ServeState;

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    gs::Seg *segs = nullptr;                 // the graph's own segment table
};

struct gs_ctx {
    gs_options opt;
    bool auto_cap = false;                   // lds_cap left to the library: sized per round by tuning_for
    size_t lds_limit = 65536;                // LDS bytes a block may use on the device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    uint64_t budget = 0;
    std::vector<uint8_t> cell_k;
    std::vector<uint64_t> cell_truth;
    std::vector<Design *> designs;
    std::vector<Stim *> stims;
    WindowBufs win;
    std::vector<LastWindow> last;            // the windows of the last round, readable by gs_read_waveform
    gs::Seg *d_segs = nullptr;
    size_t segs_cap = 0;
    unsigned long long *d_misc = nullptr;    // [0] unused, [1] flags x2 (u32), [2] flags, [4..] scratch counters
    unsigned long long *d_bump = nullptr;    // kMaxStripes stripe counters, kBumpStride apart
    // release of dead nets (gs_simulate with opt.release_dead): set while
    // gs_simulate runs; the region table and the regions' stripe counters
    bool releasing = false;
    bool last_released = false;              // the last round reused the space of dead nets
    gs::ArenaRegion *d_regions = nullptr;
    size_t regions_cap = 0;
    unsigned long long *d_rbump = nullptr;
    size_t rbump_cap = 0;                    // u64 counters
    std::vector<hipEvent_t> events;
    gs_stats stats{};
    // captured rounds, keyed by everything their launches depend on
    std::map<std::string, GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;        // library stream that graphs are captured on and launched from
    int32_t *d_c0 = nullptr;                 // first cycle of every piece of the running round
    size_t c0_cap = 0;
    // set while gs_cycle_profile runs: per-cycle totals (either may be null)
    unsigned long long *d_profile = nullptr; // glitch toggles
    unsigned long long *d_late = nullptr;    // late nets
    const int32_t *d_wout = nullptr;         // per net: slowest fanout wire, rise and fall (null: no wires)
    int32_t profile_begin = 0;               // the cycle of entry 0
    // this GPU's static scratch (gs_simulate_noalloc); while noalloc is set,
    // every device allocation the library would make fails instead
    char *d_scratch = nullptr;
    bool noalloc = false;
    std::map<std::string, std::array<int32_t, 3>> tuned;   // autotuned (cap, wpb, tpw) per batch shape
    // serving
    ServeState *serve = nullptr;
    bool serving = false;
};

gs_status gs_fail(gs_ctx *ctx, gs_status code, const char *fmt, ...);
uint64_t gs_now_ns();
void gs_dev_free(void *p);
void gs_window_release(gs_ctx *ctx, WindowBufs *w);
gs_status gs_window_reserve(gs_ctx *ctx, WindowBufs *w, uint64_t n_chunks, uint64_t words);
uint64_t gs_header_bytes(uint64_t n_nets, int32_t cycles);
uint64_t gs_arena_guess(uint64_t n_nets, int32_t cycles, int64_t toggles);
gs_status gs_check_ranges(gs_ctx *ctx, const Design *d, const Stim *s, int32_t b, int32_t e);
// Converts the segment range [b, e) of a continuous view into its cycle
// range (other stimuli: unchanged).
gs_status gs_job_cycles(gs_ctx *ctx, int32_t stim, int32_t &b, int32_t &e);
gs::WinView gs_make_view(gs_ctx *ctx, const WindowBufs &w, int32_t cycles, int32_t period, uint64_t chunk_base,
                         uint64_t n_chunks_used);
gs_status gs_ensure_segs(gs_ctx *ctx, size_t n);
hipEvent_t gs_event(gs_ctx *ctx, size_t i);
void gs_serve_shutdown(gs_ctx *ctx);
Design *gs_get_design(gs_ctx *ctx, int32_t id);
void gs_graph_cache_clear(gs_ctx *ctx);
