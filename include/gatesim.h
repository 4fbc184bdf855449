/*
 * gatesim.h — C ABI of the MI355X (gfx950) gate-level re-simulator.
 *
 * The library re-simulates combinational gate-level netlists whose input
 * waveforms (primary inputs and register/RAM outputs) are known, with
 * per-arc rise/fall gate delays, SDF-style conditional delays, optional
 * interconnect delays and inertial pulse filtering, and reduces the result
 * to SAIF-style per-net toggle counts and time-at-0/1.  This is the method
 * of GATSPI (Zhang, Ren, Sridharan, Khailany, DAC 2022): re-simulation with
 * the cycle-to-cycle dependency broken by the known sequential waveforms
 * (Section 1), levelized evaluation with every gate of a level and every
 * cycle simulated in parallel (Section 3), and the per-gate, per-cycle
 * waveform algorithm of Algorithm 1.
 *
 * Conventions for every call:
 *  - Every function returns a gs_status; nothing throws or aborts across
 *    the ABI.  On failure gs_last_error() describes the cause.
 *  - Input arrays are host pointers, borrowed for the duration of the call
 *    only (copied or uploaded before return).  Output arrays are host
 *    pointers owned by the caller.
 *  - Device memory belongs to the context, or to the caller's arena when
 *    gs_options.arena is set (the caller keeps it alive until gs_destroy).
 *  - All times are integer picoseconds; counts and SAIF sums are int64.
 *  - A context is used by one host thread at a time, except gs_submit,
 *    gs_poll and gs_release, which are thread-safe.
 *
 * Semantics (the "cycle-isolated" model of re-simulation; GATSPI Section 1
 * and Section 3, Algorithm 1):
 *  - Cycle c covers absolute times [c*T, (c+1)*T) and is simulated on its
 *    own in local time t = absolute - c*T.  At t = 0 each input holds its
 *    value from just before c*T and every net holds the zero-delay settled
 *    value (Algorithm 1, initial value).  The cycle runs to quiescence;
 *    edges later than T count toward the cycle's TC but T0/T1 only measure
 *    [0, T).
 *  - Interconnect filter (Algorithm 1, net-delay filtering): a net pulse
 *    narrower than the wire delay of its leading edge never reaches the pin.
 *  - Multiple simultaneous inputs (Algorithm 1, MSI resolution): pins
 *    switching at the same time are applied together; the output edge takes
 *    the smallest of their arc delays, looked up in the pin state after the
 *    switch.
 *  - Delay lookup (Algorithm 1's delay rows, indexed by input and output
 *    edge; SDF conditional and posedge/negedge records): in each pin state
 *    the most specific matching record applies (gs_arc).
 *  - Gate inertial filter with PATHPULSEPERCENT = 100 (Algorithm 1, output
 *    filter): when the output must change while its previous edge is still
 *    pending, the pending edge is cancelled; otherwise a new edge is
 *    scheduled after the arc delay.
 *  - SAIF (Section 3): TC = edges of the net, T1/T0 = time at 1/0, summed
 *    over the simulated cycles; IG = glitch toggles, a cycle's edges beyond
 *    its one functional edge (gs_read_saif_ig).
 *  - Optional: several cycles as one continuous segment
 *    (gs_segment_stimulus: one lane per segment; gs_continuous_stimulus:
 *    one lane per cycle with carried state); per-cycle glitch totals and a per-cycle check
 *    of when the isolated model equals a continuous run (gs_cycle_profile).
 */
#ifndef GATESIM_H
#define GATESIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs_status;
#define GS_OK           0
#define GS_E_INVALID   -1   /* malformed argument or input data */
#define GS_E_NOT_DAG   -2   /* the netlist has a combinational cycle */
#define GS_E_NOMEM     -3   /* the memory budget cannot hold one tile of one window */
#define GS_E_DEVICE    -4   /* a HIP runtime call failed or no GPU is present */
#define GS_E_STATE     -5   /* call out of order (e.g. simulate before arcs) */
#define GS_E_BUSY      -6   /* serving admission queue is full */
#define GS_E_CAPACITY  -7   /* more than 32767 transitions in one net's 64-cycle tile */

typedef struct gs_ctx gs_ctx;

/* Level schedules of the gate-evaluation kernel. */
#define GS_SCHED_LEVELS 0   /* one launch per logic level (GATSPI's level partition, Section 3) */
#define GS_SCHED_GRAPH  1   /* the same launches captured once into a HIP graph and replayed per window */

typedef struct {
    int32_t  device;          /* HIP device ordinal */
    void    *stream;          /* hipStream_t to run on, borrowed (e.g. torch's current stream); NULL = own stream */
    uint64_t hbm_budget;      /* bytes of device memory the context may hold for waveforms; 0 = 80% of free memory */
    void    *arena;           /* optional caller-owned device buffer used for all waveform storage */
    uint64_t arena_bytes;
    int32_t  window_cycles;   /* cycles per window; 0 = as many as fit the budget, capped at 16384 */
    int32_t  lds_cap;         /* transitions per (net, cycle) staged on chip by the per-tile walk (tile groups
                                 too large for the on-chip stage, cells of four or more pins, overflowing
                                 queues) before its spill path: 4, 8, 16, 24 or 32;
                                 0 = chosen per round from the input toggles per (input, cycle), or the
                                 transitions per (net, cycle) the design showed in its last round if higher:
                                 8 up to 0.5, 16 up to 1, 24 up to 3, else 32 (segment views carry many cycles per lane,
                                 glitch-heavy logic multiplies its inputs' toggles); serving uses 8 */
    int32_t  waves_per_block; /* 1, 2, 4 or 8; 0 = 4 */
    int32_t  schedule;        /* GS_SCHED_LEVELS or GS_SCHED_GRAPH */
    int32_t  timing;          /* nonzero: time every gate-evaluation launch with HIP events (gs_get_stats) */
    int32_t  tiles_per_wave;  /* consecutive 64-cycle tiles of one gate evaluated by one wave; 0 = 8 */
    int32_t  autotune;        /* nonzero: gs_simulate_batch picks lds_cap, waves_per_block and tiles_per_wave by
                                 timing candidates on the batch, each job cut to 2,048 cycles (once per batch
                                 shape; another setting must beat the default by 3%) */
    int32_t  wire_transport;  /* nonzero: interconnect delays without the net-delay filter (the paper's feature
                                 study, Section 5, Table 7, deletes Algorithm 1's filtering lines and keeps the
                                 delays): every net edge reaches the pin at its time plus the wire delay of its
                                 direction, and a pulse vanishes only when its delayed trailing edge arrives no
                                 later than its delayed leading edge; 0 = the inertial filter */
    int32_t  release_dead;    /* nonzero: gs_simulate keeps a net's transitions only until the last level that
                                 reads them (Section 3's preallocated waveform memory, with the space of dead
                                 nets reused): the window's arena is split into one region per such level,
                                 placed by the host so that a region is reused only after its level has run,
                                 and sized from the design's learned density (a region that fills up is grown
                                 and the round rerun).  Lets a window hold more cycles for the same budget;
                                 gs_read_waveform and gs_cycle_profile then refuse the call (GS_E_STATE,
                                 GS_E_INVALID), and gs_simulate_batch, gs_simulate_noalloc and serving keep
                                 every net.  0 = every net stays until the window ends */
    int32_t  reserved[3];
} gs_options;

/* Fills *opt with the defaults above. */
void gs_default_options(gs_options *opt);

/* Creates a context on opt->device (opt may be NULL for defaults): the
 * device memory the netlists, delay tables and waveforms live in, and the
 * stream the work runs on (the paper keeps the design and one preallocated
 * waveform chunk resident in GPU memory, Section 3).  Errors: GS_E_DEVICE
 * if the device cannot be used, GS_E_INVALID. */
gs_status gs_create(const gs_options *opt, gs_ctx **out);

/* Frees every device buffer of the context (not a caller-owned arena) and
 * its streams; a serving loop still running is stopped first.  NULL is a
 * no-op.  (Resource management of this library; no passage of the paper.) */
gs_status gs_destroy(gs_ctx *ctx);

/* Message for the last failure of ctx, or of a context-free call on this
 * thread when ctx is NULL.  Valid until the next call on the same ctx.
 * (Error reporting of this library; no passage of the paper.) */
const char *gs_last_error(gs_ctx *ctx);

/* Cell library (Algorithm 1's truth table Y[2^n]): cell c has n_pins[c]
 * inputs (1..6) and output bit b of truth[c] for input index b, pin 0 being
 * the least significant bit of b.  Replaces any previous library; designs
 * loaded earlier keep theirs. */
gs_status gs_load_cells(gs_ctx *ctx, int32_t n_cells, const uint8_t *n_pins, const uint64_t *truth);

/* Netlist (Section 3: the gate-level netlist as a graph).  Nets 0..n_inputs-1
 * are inputs; gate g drives net n_inputs + g.  Gate g's pins are
 * fanin_net[fanin_ptr[g] .. fanin_ptr[g+1]) in pin order; their number must
 * equal the cell's pin count and a gate's fanin nets may repeat.  The
 * netlist is levelized on the GPU (level 0 = inputs, a gate's level = 1 +
 * the largest fanin level).  Errors: GS_E_INVALID (ids out of range, arity
 * mismatch), GS_E_NOT_DAG.  *design_id receives the new design's id. */
gs_status gs_load_netlist(gs_ctx *ctx, int32_t n_inputs, int32_t n_gates, const int32_t *cell_of_gate,
                          const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t *design_id);

/* One SDF-style delay arc (Algorithm 1's per-pin gate delay table, whose
 * rows are indexed by input edge and output edge; Section 3 on conditional
 * delay statements): the delay from pin `pin` of `gate` to the output for
 * a rising (rise_ps) and a falling (fall_ps) output edge.  Two optional
 * qualifiers restrict where a record applies:
 *   cond_pin >= 0: only while pin cond_pin of the same gate has value
 *                  cond_val (read after the switch); cond_pin < 0: always;
 *   in_edge:       0 either input edge, 1 only when `pin` rises, 2 only when
 *                  it falls (SDF posedge / negedge IOPATH rows).
 * In each pin state the matching record with the most qualifiers wins.
 * 16 bytes, natural alignment. */
typedef struct {
    int32_t gate;
    int8_t  pin;
    int8_t  cond_pin;
    int8_t  cond_val;
    int8_t  in_edge;
    int32_t rise_ps;
    int32_t fall_ps;
} gs_arc;

/* Delay arcs of a design.  For every (gate, pin, pin state after the
 * switch) exactly one record of the highest matching specificity must
 * exist (records fully covered by more specific ones may repeat); all
 * conditional records of one (gate, pin) must key on the same condition
 * pin.  Delays are either all >= 1, or all 0 together with all wire delays
 * (zero-delay mode).  Replaces earlier arcs of the design.
 * Errors: GS_E_INVALID. */
gs_status gs_load_arcs(gs_ctx *ctx, int32_t design, int64_t n_arcs, const gs_arc *arcs);

/* Interconnect delays (Algorithm 1's per-pin wire delays), one rise/fall
 * pair per fanin slot in CSR order; NULL pointers mean all zero.  Each pair
 * is both 0 or both >= 1.  Errors: GS_E_INVALID. */
gs_status gs_load_wires(gs_ctx *ctx, int32_t design, const int32_t *rise_ps, const int32_t *fall_ps);

/* Input waveforms (the known primary/pseudo-primary waveforms of
 * re-simulation, Section 1): input i starts at init[i] (0/1) and toggles at
 * the absolute times toggle_ps[toggle_ptr[i] .. toggle_ptr[i+1]), strictly
 * increasing, within [0, n_cycles * period_ps).  period_ps <= 2^24.
 * Uploaded to the device.  Errors: GS_E_INVALID.  *stim_id receives the id. */
gs_status gs_load_stimulus(gs_ctx *ctx, int32_t design, int32_t period_ps, int32_t n_cycles,
                           const uint8_t *init, const int64_t *toggle_ptr, const int64_t *toggle_ps,
                           int32_t *stim_id);

/* Per-cycle glitch profile, whose peaks are the glitch hot spots that the
 * glitch-optimization flow of Section 4 targets: re-simulates cycles
 * [cycle_begin, cycle_end) exactly as gs_simulate does (adding the SAIF
 * counts) and writes into per_cycle[c - cycle_begin] the glitch toggles of
 * cycle c summed over all nets of the design (each net's edge count in the
 * cycle less its parity; summed over the range it equals the sum of
 * gs_read_saif_ig's per-net glitch toggles).  per_cycle: caller-owned host
 * array of cycle_end - cycle_begin entries.  Costs one extra pass over each
 * window's per-lane edge counts (2 bytes per net and cycle) and a small
 * device allocation per call.  Errors: as gs_simulate. */
gs_status gs_glitch_profile(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end,
                            int64_t *per_cycle);

/* Per-cycle profile with a check of the cycle-isolated reading (Section 1
 * breaks the cycle dependency with known waveforms; that is exact where
 * logic settles within a period): re-simulates [cycle_begin, cycle_end) as
 * gs_simulate does (adding the SAIF counts) and writes, for every cycle c of
 * the range at index c - cycle_begin,
 *   glitch[]: the glitch toggles of cycle c over all nets (gs_glitch_profile);
 *   late[]:   the nets whose last edge in cycle c, or that edge's arrival at
 *             a fanout pin through the net's slowest wire for the edge's
 *             direction, lies at or after the period.
 * A cycle with no late net ends quiescent, so the next cycle's isolated
 * start is exactly the state a continuous run reaches: when no cycle but
 * the last of a range has a late net, the range's cycle-by-cycle result
 * equals one continuous run over it.  The test is conservative (such an
 * arrival may still be filtered out).  On a segment view, cycles are
 * segments.  Either array may be NULL; both are caller-owned host arrays of
 * cycle_end - cycle_begin entries.  The late count reads one extra word per
 * (net, cycle) that has edges.  Errors: as gs_simulate. */
gs_status gs_cycle_profile(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end,
                           int64_t *glitch, int64_t *late);

/* Continuous segments (the re-simulation of Section 1 without isolating
 * every cycle): creates a view of stimulus `stim` in which each group of
 * segment_cycles consecutive cycles, from cycle 0, is one cycle.  Every call
 * that takes the new id then runs each group as one continuous simulation
 * from the settled state at its start, so edges and pending events cross
 * the cycle boundaries inside it.  Cycle indices, waveform readback and
 * T0/T1 count segments; the glitch toggles of gs_read_saif_ig count each
 * segment's edges beyond its net value change (an upper bound on its
 * glitches).  The view shares the device arrays of `stim`.  Needs n_cycles
 * to be a multiple of segment_cycles and segment_cycles x period_ps <= 2^24.
 * Errors: GS_E_INVALID.  *stim_id receives the new id. */
gs_status gs_segment_stimulus(gs_ctx *ctx, int32_t stim, int32_t segment_cycles, int32_t *stim_id);

/* Continuous segments with cycle-parallel lanes (Section 1's re-simulation
 * of known waveforms, run with Section 3's one thread per cycle): a view of
 * stimulus `stim` with the same results as gs_segment_stimulus's view of the
 * same segment_cycles, but every cycle of a segment keeps a lane of its own.
 * A lane's list holds the edges before the end of its cycle; the output edge
 * still pending there (at most one) is carried into the next cycle of the
 * segment, which then starts with it pending, and lanes are evaluated
 * again until no carry changes; the last cycle of a segment keeps all its
 * edges.  Cycle indices of calls that take the view count segments, as for
 * gs_segment_stimulus; gs_read_waveform returns a segment's edges in segment
 * time.  Windows hold whole segments (GS_E_NOMEM if one segment does not
 * fit the budget).  Runs through gs_simulate, gs_simulate_noalloc and
 * gs_simulate_batch, for designs without interconnect delays; gs_autotune,
 * gs_cycle_profile and serving reject it (GS_E_INVALID).  `stim` must not be
 * a view.  Needs n_cycles to be a multiple of segment_cycles.  Errors:
 * GS_E_INVALID.  *stim_id receives the new id. */
gs_status gs_continuous_stimulus(gs_ctx *ctx, int32_t stim, int32_t segment_cycles, int32_t *stim_id);

/* Re-simulates cycles [cycle_begin, cycle_end) of stimulus `stim` on
 * `design` and ADDS the per-net SAIF counts into the design's accumulators.
 * The range is processed in windows that fit the memory budget; under the
 * cycle-isolated model the result does not depend on the window size.
 * Synchronous: returns after the device work is complete.  Errors:
 * GS_E_STATE (no arcs), GS_E_INVALID (range), GS_E_NOMEM, GS_E_CAPACITY,
 * GS_E_DEVICE. */
gs_status gs_simulate(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * re-simulation and SAIF accumulation as gs_simulate, with the same result,
 * but every device buffer the call needs beyond the loaded design and
 * stimulus (window chunk headers, lane ends and transition arena, flags,
 * stripe counters, the level segment table) lives in a static device array
 * of GS_SCRATCH_BYTES per GPU, which the library holds from gs_create until
 * the process ends.  The call makes no device allocation and no graph
 * capture; it runs direct launches on the context's stream, synchronously.
 * Windows are as long as their chunk headers and lane ends fit in half of the
 * scratch, and are halved when the transition arena fills up.  Calls on one
 * GPU share its scratch, which keeps the last call's contents: calls that
 * overlap on one GPU (other threads or contexts) race.  gs_read_waveform
 * does not see windows run by this call.  Errors: as gs_simulate, and
 * GS_E_NOMEM when a 64-cycle window of the design (144 bytes per net) or its
 * levels (at most 5,957) do not fit the scratch. */
#define GS_SCRATCH_BYTES (64ull << 20)
gs_status gs_simulate_noalloc(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end);

/* Copies the design's accumulated SAIF counts, n_inputs + n_gates entries
 * each, into caller arrays (any may be NULL); nonzero reset zeroes the
 * accumulators afterwards.  Page-locked arrays (hipHostMalloc) are filled
 * by one DMA each; pageable ones are staged by the HIP runtime, which is
 * several times slower for large designs. */
gs_status gs_read_saif(gs_ctx *ctx, int32_t design, int64_t *tc, int64_t *t0, int64_t *t1, int32_t reset);

/* As gs_read_saif, and also the glitch toggles per net (SAIF's IG; the
 * paper's SAIF output, Section 3): a cycle whose list has L edges adds
 * L - (L mod 2), every edge but the one functional edge of an odd list.
 * Any array may be NULL; reset zeroes all four accumulators. */
gs_status gs_read_saif_ig(gs_ctx *ctx, int32_t design, int64_t *tc, int64_t *t0, int64_t *t1, int64_t *ig,
                          int32_t reset);

/* Debug/spot-check read of one net's waveform in one cycle of the most
 * recently simulated window of (design, stim): the output list Algorithm 1
 * writes for a (net, cycle), as its initial value and edge times.  *init
 * gets the value at t = 0, *n the number of edges, times[0 .. min(*n, cap))
 * the edge times in cycle-local ps.  GS_E_STATE if the cycle is not
 * resident (windows of gs_simulate_noalloc and of the batch and serving
 * calls are not kept). */
gs_status gs_read_waveform(gs_ctx *ctx, int32_t design, int32_t stim, int32_t net, int32_t cycle,
                           int32_t *init, int32_t *times, int32_t cap, int32_t *n);

typedef struct {
    int32_t n_inputs, n_gates, n_levels, max_pins;
    int64_t n_fanin;
    int32_t has_wires, zero_delay;
    int32_t max_delay_ps, reserved;
} gs_design_info;

gs_status gs_get_design_info(gs_ctx *ctx, int32_t design, gs_design_info *info);

/* Level of every gate (n_gates entries) as computed by the GPU levelizer. */
gs_status gs_get_levels(gs_ctx *ctx, int32_t design, int32_t *level);

typedef struct {
    double   gate_eval_ms;      /* summed HIP-event time of gate-evaluation launches (timing on) */
    double   expand_ms;         /* summed time of stimulus-expansion launches (timing on) */
    double   wall_ms;           /* host wall time inside gs_simulate / gs_simulate_batch */
    int64_t  gate_eval_launches;
    int64_t  windows;
    int64_t  window_retries;    /* windows redone after the transition arena filled up */
    int64_t  gate_cycles;       /* gates x cycles simulated */
    int64_t  spilled_lanes;     /* (net, cycle) lists longer than the on-chip staging cap */
    int64_t  arena_words;       /* 32-bit transition slots used by the last window */
    int64_t  graph_launches;    /* rounds replayed from a captured HIP graph */
    int64_t  unstaged_groups;   /* (gate, tile group) waves whose fanin words exceeded the on-chip stage */
    int64_t  queue_overflows;   /* staged tile groups of gates with up to three pins that had more lanes with
                                   two or more pin events than the compacted walk queues, and took the per-tile
                                   walk instead */
    int64_t  release_peak_words; /* with release_dead: arena words the last round's regions took at their peak
                                   (arena_words counts every transition the round stored) */
    int64_t  reserved[2];
} gs_stats;

gs_status gs_get_stats(gs_ctx *ctx, gs_stats *st, int32_t reset);

/* ---------------------------------------------------------------------
 * Host-only checks (no device needed): the validation that the load calls
 * run before touching the GPU, exposed for callers and tests.
 * ------------------------------------------------------------------- */
gs_status gs_check_netlist(int32_t n_cells, const uint8_t *n_pins, int32_t n_inputs, int32_t n_gates,
                           const int32_t *cell_of_gate, const int64_t *fanin_ptr, const int32_t *fanin_net);
gs_status gs_check_arcs(int32_t n_cells, const uint8_t *n_pins, int32_t n_gates, const int32_t *cell_of_gate,
                        int64_t n_arcs, const gs_arc *arcs);
gs_status gs_check_stimulus(int32_t n_inputs, int32_t period_ps, int32_t n_cycles, const uint8_t *init,
                            const int64_t *toggle_ptr, const int64_t *toggle_ps);

/* ---------------------------------------------------------------------
 * Batching: many (design, stimulus, cycle range) jobs of uneven sizes in
 * one schedule.  Level k of every job is evaluated by one launch over a
 * work list of (job, gate, cycle tile) items; the launch sequence of a
 * batch composition is captured into a HIP graph and replayed.  Per-job
 * results are identical to running each job alone with gs_simulate; SAIF
 * counts are added into each job's design accumulators.
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t design;
    int32_t stim;
    int32_t cycle_begin;
    int32_t cycle_end;
} gs_job;

/* Runs the jobs as rounds that fit the memory budget; level k of every job
 * of a round is one launch, and a round's launches are replayed from a
 * captured HIP graph when the schedule is GS_SCHED_GRAPH.  The paper runs
 * one design per invocation and pays a stream synchronisation and kernel
 * launch per level (Section 5, Table 5); batching shares those costs among
 * the jobs.  Errors: as gs_simulate for each job (checked before any work). */
gs_status gs_simulate_batch(gs_ctx *ctx, int32_t n_jobs, const gs_job *jobs);

/* Autotuner: times candidate (lds_cap, waves_per_block, tiles_per_wave)
 * settings of the gate-evaluation kernel on cycles [cycle_begin, cycle_end)
 * (at most 4096) of (design, stim), with nothing added to the SAIF
 * accumulators, and keeps the fastest in the context's options.  The paper
 * tunes its cycle parallelism and threads per block by measurement
 * (Section 5, Table 6); these are the corresponding knobs here. */
typedef struct {
    int32_t lds_cap, waves_per_block, tiles_per_wave, reserved;
    double  trial_ms;           /* gate-evaluation time of the winning setting on the trial */
} gs_tuning;

gs_status gs_autotune(gs_ctx *ctx, int32_t design, int32_t stim, int32_t cycle_begin, int32_t cycle_end,
                      gs_tuning *out);

/* ---------------------------------------------------------------------
 * Serving: a resident request loop with continuous batching (the
 * re-simulation step of GATSPI's glitch-optimization flow, Section 4).
 * Requests are admitted while their device-memory footprint fits the free
 * budget; admitted requests join the running level schedule at the next
 * step, so their work overlaps on the device.
 * ------------------------------------------------------------------- */
#define GS_REQ_WINDOW 0     /* re-simulate cycles [cycle_begin, cycle_end) of (design, stim) */
#define GS_REQ_EDIT   1     /* re-simulate the resident window with edited delay arcs */

typedef struct {
    int32_t gate;
    int8_t  pin;
    int8_t  cond_pin;       /* with cond_val and in_edge, selects the record being edited */
    int8_t  cond_val;
    int8_t  in_edge;
    int32_t rise_ps;        /* new delays */
    int32_t fall_ps;
} gs_arc_edit;

typedef struct {
    int32_t kind;           /* GS_REQ_WINDOW or GS_REQ_EDIT */
    int32_t design;
    int32_t stim;
    int32_t cycle_begin;    /* GS_REQ_WINDOW */
    int32_t cycle_end;
    int32_t n_edits;        /* GS_REQ_EDIT */
    const gs_arc_edit *edits;
} gs_request;

typedef struct {
    int32_t  status;        /* GS_OK, or the request's error */
    int32_t  n_nets;
    const int64_t *tc;      /* library-owned until gs_release(ticket) */
    const int64_t *t0;
    const int64_t *t1;
    const int64_t *ig;      /* glitch toggles, as gs_read_saif_ig */
    int64_t  gate_cycles;   /* gates x cycles re-simulated for this request */
    uint64_t t_submit_ns;   /* CLOCK_MONOTONIC */
    uint64_t t_admit_ns;
    uint64_t t_done_ns;
} gs_result;

/* Starts the serving loop: `resident_cycles` cycles starting at
 * resident_begin of (design, stim) pairs given are simulated once and kept
 * on the device as the base that delay-edit requests re-simulate against.
 * max_queue bounds waiting requests (GS_E_BUSY beyond it). */
gs_status gs_serve_start(gs_ctx *ctx, int32_t n_resident, const int32_t *designs, const int32_t *stims,
                         const int32_t *resident_begin, const int32_t *resident_cycles, int32_t max_queue);
gs_status gs_submit(gs_ctx *ctx, const gs_request *req, uint64_t *ticket);
/* Non-blocking unless wait is nonzero.  Returns GS_E_BUSY while pending. */
gs_status gs_poll(gs_ctx *ctx, uint64_t ticket, int32_t wait, gs_result *res);
gs_status gs_release(gs_ctx *ctx, uint64_t ticket);
gs_status gs_serve_stop(gs_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GATESIM_H */
