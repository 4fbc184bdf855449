// Internal structures shared by the host core (host.cpp) and the gfx950
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

constexpr int kLanes = 64;                  // wavefront size on CDNA; one lane per cycle of a tile
constexpr int32_t kInf = 0x7fffffff;        // end-of-waveform time (Algorithm 1's EOW)
// A lane end is 16 bits: the inclusive transition count of the chunk up to
// that lane (15 bits) and, in bit 15, the net's value at the start of the
// lane's cycle.
constexpr uint32_t kMaxChunk = 32767;       // transitions per (net, 64-cycle tile)
constexpr uint32_t kEndCount = 0x7fffu;
constexpr uint32_t kEndInitShift = 15;

// Fanin words a gate-evaluation wave stages in LDS for one group of tiles.
constexpr uint32_t kStageWords = 512;

// Compacted evaluation of a staged tile group: a lane never has more output
// edges than pin events, so the group's output edges fit a stage of the
// same size; lanes with two or more pin events are queued (up to
// kQueueCap of them, one word per pin, at most kQueueWords) and walked
// together.
constexpr uint32_t kOutStageWords = kStageWords;
constexpr uint32_t kQueueCap = 192;
constexpr uint32_t kQueueWords = 3;

// LDS words of one gate-evaluation wave: the delay table (64 words), the
// fanin stage, then a region shared by the per-lane output slots of the
// per-tile path (cap + 1 per lane) and the output stage plus lane queue of
// the compacted path.
__host__ __device__ constexpr size_t gate_eval_wave_words(int cap)
{
    return (size_t)kLanes + kStageWords +
           ((size_t)(cap + 1) * kLanes > (size_t)kOutStageWords + kQueueCap * kQueueWords
                ? (size_t)(cap + 1) * kLanes
                : (size_t)kOutStageWords + kQueueCap * kQueueWords);
}

__host__ __device__ constexpr size_t gate_eval_lds_bytes(int cap, int wpb)
{
    return (size_t)wpb * gate_eval_wave_words(cap) * sizeof(int32_t);
}

// One gate in level order (the level partition of Section 3), 32 bytes.
struct GateRec {
    uint32_t out;       // output net id
    uint32_t pin0;      // index of its first PinRec
    uint32_t k;         // number of pins
    uint32_t dead;      // the output's arena region when dead nets are released (by its level and the
                        // last level that reads it)
    uint64_t truth;     // truth bits, pin 0 = least significant bit of the index
    uint64_t pad2;
};

// Index into a pin's delay row: cv = value of the row's condition pin q,
// ie = 1 for a rising input edge, oe = 1 for a rising output edge, all read
// in the gate's pin state after the switch (ie is the pin's own bit there).
__host__ __device__ constexpr int delay_slot(int cv, int ie, int oe) { return (cv << 2) | (ie << 1) | oe; }

// One gate pin (fanin arc), 48 bytes: its net, the condition pin q of its
// delay row, the row d[delay_slot(cv, ie, oe)] and its interconnect delays.
struct PinRec {
    int32_t net;
    int32_t q;
    int32_t d[8];
    int32_t wr, wf;     // interconnect rise / fall delay
};

// Where the transitions of one (net, 64-cycle tile) live: `off` is the word
// offset of the chunk in the window's transition arena; bit l of `mask` is
// the value of the net at t = 0 of the tile's cycle l.
struct ChunkHdr {
    uint64_t off;
    uint64_t mask;
};

// One region of a window's transition arena when dead nets are released:
// the chunks of nets written by one level and last read by about the same
// level (region 0: the inputs), with its own stripe counters.  The host
// places regions so that one is reused only after its last reader has run.
struct ArenaRegion {
    uint64_t off;                  // first word, counted from `times`
    uint64_t slice_words;          // words per stripe
    unsigned long long *bump;      // its stripe counters, kBumpStride apart
    uint32_t stripe_mask;
    uint32_t pad;
};

// A window of cycles resident on the device.
//   hdr[net * n_tiles + tile]
//   ends[(net * n_tiles + tile) * 64 + lane]: inclusive prefix sum of the
//     per-cycle transition counts inside the chunk
//   times[hdr.off + ...]: cycle-local transition times, lane after lane
struct WinView {
    ChunkHdr *hdr;
    uint16_t *ends;
    int32_t *times;
    unsigned long long *bump;      // per stripe, kBumpStride apart: [0] words taken from the stripe (by handed-out
                                   // reservations and failed tries), [1] words of failed tries
    unsigned int *flags;           // [0] arena full, [1] chunk over kMaxChunk, [2] spilled lanes, [3] bound violated,
                                   // [4] tile groups walked from the arena (too many words to stage),
                                   // [5] staged groups whose multi-event lanes overflowed the compacted queue
    uint64_t slice_words;          // arena words owned by each stripe
    uint64_t arena_off;            // first word of this window's arena, counted from `times`
    int32_t n_tiles;
    int32_t n_cycles;              // cycles in this window
    int32_t period;
    uint32_t stripe_mask;          // stripes - 1 (a power of two)
    // Cone re-simulation: when `slot` is set, net n's chunks live at slot[n]
    // of hdr/ends if slot[n] >= 0 (a re-simulated net) and otherwise at n of
    // rd_hdr/rd_ends (the resident window the cone is evaluated against).
    const int32_t *slot;
    const ChunkHdr *rd_hdr;
    const uint16_t *rd_ends;
    // Release of dead nets: when set, region GateRec::dead of this table
    // (region 0 for the inputs) replaces arena_off, slice_words, bump and
    // stripe_mask for a producer's reservations.
    const ArenaRegion *regions;
};

// The transition arena is split into stripes, each with its own bump
// counter on its own 256-byte line, so that the per-wave reservations of a
// launch spread over many addresses instead of serialising on one.
constexpr int kMaxStripes = 512;
constexpr int kBumpStride = 32;             // u64 counters between stripes (256 B)

// SAIF accumulators, N entries each and contiguous in this order: toggle
// count, time at 0, time at 1, glitch toggles (edges of a cycle beyond its
// functional one).
constexpr int kSaifArrays = 4;
struct SaifAcc {
    unsigned long long *tc;
    unsigned long long *t0;
    unsigned long long *t1;
    unsigned long long *ig;
};

// The accumulators of N nets starting at base.
inline SaifAcc saif_view(unsigned long long *base, size_t n)
{
    return SaifAcc{base, base + n, base + 2 * n, base + 3 * n};
}

// One piece of a gate-evaluation launch: the gates [gate_begin,
// gate_begin + n_gates) of one level of one instance, all tiles of its
// window.  Wave w of the launch belongs to the segment whose
// [wave_begin, wave_begin + n_gates * n_tiles) holds it.
struct Seg {
    uint64_t wave_begin;
    const GateRec *gates;
    const PinRec *pins;
    uint32_t gate_begin;
    uint32_t n_gates;
    uint32_t salt;                 // added to the block index to pick an arena stripe
    uint32_t mode;                 // bit 0: transport wire delays (no net-delay filter); bits 8-31: cycles of a
                                   // continuous segment whose cycles are lanes (0: every cycle on its own)
    WinView win;
    SaifAcc saif;
};

// Device copy of one stimulus.
struct StimView {
    const uint8_t *init;
    const int64_t *toggle_ptr;
    const int64_t *toggle_ps;
    int32_t n_inputs;
    int32_t period;
    int32_t seg;        // > 1: glitch toggles counted per continuous segment of this many cycles
};

// Static device scratch of gs_simulate_noalloc (bytes per GPU), and the
// devices whose scratch address is kept.
constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

// Address of this GPU's static scratch: looked up with hipGetSymbolAddress
// on the first call for a device, which must be the current device then,
// and kept for later calls.
hipError_t scratch_region(int device, void **ptr);

// ---- launchers (kernels.hip) ------------------------------------------
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u32(unsigned int *p, uint64_t n, unsigned int v, hipStream_t s);
hipError_t launch_add_u64(unsigned long long *dst, const unsigned long long *src, uint64_t n, hipStream_t s);
hipError_t launch_add_u64_guarded(unsigned long long *dst, const unsigned long long *src, uint64_t n,
                                  const unsigned int *flags, hipStream_t s);

hipError_t launch_level_init(int32_t *level, int32_t n_inputs, int32_t n_gates, hipStream_t s);
hipError_t launch_fanout_count(const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t n_inputs, int32_t n_gates,
                               unsigned int *pending, unsigned int *fo_cnt, hipStream_t s);
hipError_t launch_fanout_fill(const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t n_inputs, int32_t n_gates,
                              const int64_t *fo_ptr, unsigned int *cursor, int32_t *fo, hipStream_t s);
hipError_t launch_level_seed(const unsigned int *pending, int32_t *level, int32_t n_inputs, int32_t n_gates,
                             int32_t *frontier, unsigned int *size, hipStream_t s);
hipError_t launch_level_frontier(const int32_t *frontier, unsigned int n, const int64_t *fo_ptr, const int32_t *fo,
                                 const int64_t *fanin_ptr, const int32_t *fanin_net, unsigned int *pending,
                                 int32_t *level, int32_t n_inputs, int32_t *next, unsigned int *next_size,
                                 hipStream_t s);
hipError_t launch_level_bucket(const int32_t *level, int32_t n_inputs, int32_t n_gates,
                               unsigned int *cursor, int32_t *perm, int count_only, hipStream_t s);

hipError_t launch_expand(StimView st, WinView win, SaifAcc acc, const int32_t *cycle0, uint32_t salt, hipStream_t s);

// cont: every segment runs continuous segments of (mode >> 8) cycles, each
// wave's tiles starting one (no interconnect delays, no remap).
hipError_t launch_gate_eval(const Seg *segs, int32_t n_segs, uint64_t n_waves, int32_t wires,
                            int32_t cap, int32_t wpb, int32_t kmax, uint32_t tpw, int32_t remap, int32_t cont,
                            hipStream_t s);

// New delays of one edited fanin slot, addressed by (output net, pin).
struct EditRec {
    uint32_t out;
    uint32_t pin;
    int32_t d[8];       // the new delay row, as PinRec::d
};

// Fanout-cone marking for delay edits, one launch per level: mark[out] |= the
// OR of mark over the gate's fanin nets (marks of edited gates preset);
// *count counts the level's marked gates.
hipError_t launch_cone_mark(const GateRec *gates, const PinRec *pins, uint32_t gate_begin, uint32_t n_gates,
                            uint8_t *mark, unsigned int *count, hipStream_t s);
hipError_t launch_mark_set(const uint32_t *nets, uint32_t n, uint8_t *mark, hipStream_t s);
hipError_t launch_cone_place(const GateRec *gates, const PinRec *pins, uint32_t n_gates, const uint8_t *mark,
                             const int32_t *level, const unsigned int *off, unsigned int *cur, GateRec *cg, PinRec *cp,
                             uint32_t stride, int32_t *slot, uint32_t n_cone, hipStream_t s);
hipError_t launch_edit_apply(const EditRec *ed, uint32_t n, const int32_t *slot, PinRec *cp, uint32_t stride,
                             uint32_t n_cone, hipStream_t s);
// Zeroes the SAIF counters of the output nets of gates[0 .. n).
// Adds, for every cycle of a finished window, the glitch toggles of nets
// [0, n_nets) (edge count less its parity) into glitch[cycle] and, when late
// is not null, the nets whose last edge, or its arrival through the net's
// slowest fanout wire (wout: rise and fall maximum per net, null = none),
// reaches the period into late[cycle].  glitch may be null.
hipError_t launch_cycle_profile(const uint16_t *ends, const ChunkHdr *hdr, const int32_t *times, const int32_t *wout,
                                uint32_t n_nets, uint32_t tiles, uint32_t cycles, int32_t period,
                                unsigned long long *glitch, unsigned long long *late, hipStream_t s);
hipError_t launch_saif_zero(const GateRec *gates, uint32_t n, SaifAcc acc, hipStream_t s);

}  // namespace gs
