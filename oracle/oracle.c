/*
 * Reference simulator: plain, single-threaded, event-driven, 2-valued,
 * inertial-delay gate-level re-simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it; the library never does.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * What it computes (GATSPI, Section 3 and Algorithm 1, read as an event
 * simulation):
 *
 *  - Re-simulation (Section 1): input waveforms are given; only the
 *    combinational gates are simulated.  Every clock cycle is simulated on
 *    its own in cycle-local time t = absolute - c*T (the known sequential
 *    waveforms break the cycle-to-cycle dependency, Section 1 and Section 3).
 *    At t = 0 each input holds its value from just before c*T, and every
 *    gate output and gate pin holds the zero-delay settled value of those
 *    inputs (Algorithm 1, initial value).  Input toggles in [c*T, (c+1)*T)
 *    are events at their local times.  The cycle runs until no event is left;
 *    edges later than T still belong to cycle c.
 *
 *  - Interconnect (Algorithm 1, net-delay filtering): every fanin arc has a
 *    rise and a fall wire delay chosen by the value the net switches to.
 *    When the net switches at t and the arc still holds a pending pin edge at
 *    a time tp with t < tp, that pending edge is cancelled (the pulse was
 *    narrower than the wire delay of its leading edge); otherwise a pin edge
 *    is scheduled at t + delay.
 *
 *  - Interconnect without the filter (the paper's feature study, Section 5
 *    and Table 7, deletes Algorithm 1's net-delay filtering lines and keeps
 *    the wire delays): every net edge reaches the pin at t + delay, a
 *    transport delay.  Only a pulse whose delayed trailing edge would arrive
 *    no later than its delayed leading edge (possible when the rise and fall
 *    wire delays differ) vanishes: the new arrival a = t + delay cancels the
 *    arc's last scheduled pin edge when that edge is pending at a time
 *    tp >= a, and is not scheduled itself.  (Several pin edges may then be
 *    pending on one arc; the last scheduled one is the latest of them.)
 *
 *  - Multiple simultaneous inputs (Algorithm 1, MSI resolution): all pin
 *    edges of a gate at the same time are applied first, then the gate is
 *    evaluated once by truth-table lookup (pin 0 is the least significant
 *    bit of the table index).
 *
 *  - Gate delay (Algorithm 1, gate delay lookup, whose delay rows are
 *    indexed by the input edge and the output edge; Section 3 on SDF): the
 *    delay of pin j's arc for output edge e in the gate's pin state s (after
 *    the switch, so pin j's own bit gives its input edge: 1 = rising) comes
 *    from the most specific matching record.  A record may carry a condition
 *    (its condition pin has the stated value in s) and an input-edge
 *    qualifier (rising or falling input only); each qualifier it carries
 *    must hold, and its specificity is the number of qualifiers.  Exactly
 *    one record of the highest matching specificity must exist for every
 *    state.  When several pins switch together the output edge takes the
 *    smallest of their delays, looked up in the state after all of them
 *    switched.
 *
 *  - Gate inertial filter with PATHPULSEPERCENT = 100 (Algorithm 1, output
 *    filter; Section 3): after evaluation, with y the new value, z the value
 *    the output is heading to (after its pending edge, if any): if y == z
 *    nothing happens; if y != z and an edge is still pending (it lies later
 *    than t) that edge is cancelled; otherwise an edge to y is scheduled at
 *    t + delay.
 *
 *  - Same-time order: at one time t, events are handled by increasing logic
 *    level; at one level net edges come first, then pin edges, then gate
 *    evaluations.  Zero-delay designs therefore settle level by level at the
 *    same t.
 *
 *  - SAIF (Section 3): per net, TC = number of edges, T1 / T0 = time at 1 /
 *    at 0 inside [0, T) of each cycle, each summed over the cycles.
 *
 * The event queue is a binary heap of indices into an event pool; a
 * cancelled event stays in the heap and is skipped when popped.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

enum { EV_NET = 0, EV_PIN = 1, EV_EVAL = 2 };

typedef struct {
    int64_t t;
    int32_t level;
    int32_t kind;      /* also the same-time phase: net < pin < eval */
    int64_t seq;
    int32_t id;        /* net id, fanin slot, or gate */
    int32_t val;
    int32_t cancelled;
} Event;

typedef struct {
    int32_t n_inputs, n_gates, n_nets;
    int32_t *cell_pins;         /* per gate */
    uint64_t *truth;            /* per gate */
    int64_t *fanin_ptr;         /* [G+1] */
    int32_t *fanin_net;         /* [F] */
    int32_t *slot_gate;         /* [F] gate owning a fanin slot */
    int32_t *slot_pin;          /* [F] pin index of a fanin slot */
    int32_t *wire_r, *wire_f;   /* [F] */
    int64_t *fo_ptr;            /* [N+1] fanout CSR over fanin slots */
    int32_t *fo_slot;           /* [F] */
    int32_t *level;             /* per net: inputs 0, gate net 1 + max fanin level */
    int32_t *topo;              /* gates in non-decreasing level order */
    int64_t *dtab_ptr;          /* [F+1] offset into dtab, 2 entries per pin state */
    int32_t *dtab;              /* delay per (slot, state, edge): edge 0 = fall, 1 = rise */
} Design;

/* ---------------------------------------------------------------- utils */
static void set_err(char *err, int errlen, const char *msg)
{
    if (err && errlen > 0) {
        strncpy(err, msg, (size_t)errlen - 1);
        err[errlen - 1] = 0;
    }
}

void oracle_free(void *p)
{
    Design *d = (Design *)p;
    if (!d) return;
    free(d->cell_pins); free(d->truth); free(d->fanin_ptr); free(d->fanin_net);
    free(d->slot_gate); free(d->slot_pin); free(d->wire_r); free(d->wire_f);
    free(d->fo_ptr); free(d->fo_slot); free(d->level); free(d->topo);
    free(d->dtab_ptr); free(d->dtab);
    free(d);
}

/*
 * Build a design.  Arc records follow the SDF reading above: cond_pin < 0
 * means unconditional; arc_in_edge (may be NULL: all 0) is 0 for either
 * input edge, 1 for a rising, 2 for a falling input edge of the pin.
 * wire_r / wire_f may be NULL (all zero).
 * Returns NULL and fills err on bad input.
 */
void *oracle_new(int32_t n_inputs, int32_t n_gates,
                 int32_t n_cells, const uint8_t *cell_n_pins, const uint64_t *cell_truth,
                 const int32_t *cell_of_gate, const int64_t *fanin_ptr, const int32_t *fanin_net,
                 int64_t n_arcs, const int32_t *arc_gate, const int8_t *arc_pin,
                 const int8_t *arc_cond_pin, const int8_t *arc_cond_val, const int8_t *arc_in_edge,
                 const int32_t *arc_rise, const int32_t *arc_fall,
                 const int32_t *wire_rise, const int32_t *wire_fall,
                 char *err, int32_t errlen)
{
    Design *d = (Design *)calloc(1, sizeof(Design));
    int32_t G = n_gates, I = n_inputs, N = I + G;
    int64_t F = fanin_ptr[G];
    d->n_inputs = I; d->n_gates = G; d->n_nets = N;
    d->cell_pins = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G + 1));
    d->truth = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(G + 1));
    d->fanin_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(G + 1));
    d->fanin_net = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F + 1));
    d->slot_gate = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F + 1));
    d->slot_pin = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F + 1));
    d->wire_r = (int32_t *)calloc((size_t)(F + 1), sizeof(int32_t));
    d->wire_f = (int32_t *)calloc((size_t)(F + 1), sizeof(int32_t));
    d->fo_ptr = (int64_t *)calloc((size_t)(N + 1), sizeof(int64_t));
    d->fo_slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F + 1));
    d->level = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    d->topo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G + 1));
    d->dtab_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(F + 1));

    for (int32_t g = 0; g < G; g++) {
        int32_t c = cell_of_gate[g];
        if (c < 0 || c >= n_cells) { set_err(err, errlen, "cell id out of range"); oracle_free(d); return NULL; }
        d->cell_pins[g] = cell_n_pins[c];
        d->truth[g] = cell_truth[c];
        d->fanin_ptr[g] = fanin_ptr[g];
        if (fanin_ptr[g + 1] - fanin_ptr[g] != cell_n_pins[c]) {
            set_err(err, errlen, "fanin count differs from cell pin count"); oracle_free(d); return NULL;
        }
    }
    d->fanin_ptr[G] = F;
    for (int32_t g = 0; g < G; g++)
        for (int64_t s = fanin_ptr[g]; s < fanin_ptr[g + 1]; s++) {
            int32_t n = fanin_net[s];
            if (n < 0 || n >= N) { set_err(err, errlen, "fanin net out of range"); oracle_free(d); return NULL; }
            d->fanin_net[s] = n;
            d->slot_gate[s] = g;
            d->slot_pin[s] = (int32_t)(s - fanin_ptr[g]);
            if (wire_rise) { d->wire_r[s] = wire_rise[s]; d->wire_f[s] = wire_fall[s]; }
        }

    /* fanout lists */
    for (int64_t s = 0; s < F; s++) d->fo_ptr[d->fanin_net[s] + 1]++;
    for (int32_t n = 0; n < N; n++) d->fo_ptr[n + 1] += d->fo_ptr[n];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
        memcpy(fill, d->fo_ptr, sizeof(int64_t) * (size_t)(N + 1));
        for (int64_t s = 0; s < F; s++) d->fo_slot[fill[d->fanin_net[s]]++] = (int32_t)s;
        free(fill);
    }

    /* levels by Kahn's algorithm: a gate is placed once all of its fanin
       nets have a level; level = 1 + the largest fanin level */
    {
        int32_t *missing = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G + 1));
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
        int64_t qh = 0, qt = 0;
        for (int32_t g = 0; g < G; g++) missing[g] = (int32_t)(fanin_ptr[g + 1] - fanin_ptr[g]);
        for (int32_t n = 0; n < N; n++) d->level[n] = -1;
        for (int32_t i = 0; i < I; i++) { d->level[i] = 0; queue[qt++] = i; }
        for (int32_t g = 0; g < G; g++)
            if (missing[g] == 0) { d->level[I + g] = 1; queue[qt++] = I + g; }
        while (qh < qt) {
            int32_t n = queue[qh++];
            for (int64_t e = d->fo_ptr[n]; e < d->fo_ptr[n + 1]; e++) {
                int32_t s = d->fo_slot[e], g = d->slot_gate[s];
                if (--missing[g] == 0) {
                    int32_t lv = 0;
                    for (int64_t t = fanin_ptr[g]; t < fanin_ptr[g + 1]; t++)
                        if (d->level[d->fanin_net[t]] > lv) lv = d->level[d->fanin_net[t]];
                    d->level[I + g] = lv + 1;
                    queue[qt++] = I + g;
                }
            }
        }
        free(missing);
        free(queue);
        for (int32_t g = 0; g < G; g++)
            if (d->level[I + g] < 0) { set_err(err, errlen, "netlist has a combinational cycle"); oracle_free(d); return NULL; }
        /* gates sorted by level (counting sort, stable by gate id) */
        int32_t maxl = 0;
        for (int32_t g = 0; g < G; g++) if (d->level[I + g] > maxl) maxl = d->level[I + g];
        int64_t *cnt = (int64_t *)calloc((size_t)maxl + 2, sizeof(int64_t));
        for (int32_t g = 0; g < G; g++) cnt[d->level[I + g] + 1]++;
        for (int32_t l = 0; l <= maxl; l++) cnt[l + 1] += cnt[l];
        for (int32_t g = 0; g < G; g++) d->topo[cnt[d->level[I + g]]++] = g;
        free(cnt);
    }

    /* delay tables: for every fanin slot, every full pin state and both
       output edges.  Records are applied from the most specific kind (both
       qualifiers) down to unqualified ones; a state takes the first kind
       that matches it, and two records of that kind matching one state are
       an error.  Every state must be matched. */
    {
        int64_t tot = 0;
        for (int64_t s = 0; s < F; s++) {
            d->dtab_ptr[s] = tot;
            tot += 2LL << d->cell_pins[d->slot_gate[s]];
        }
        d->dtab_ptr[F] = tot;
        d->dtab = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot + 1));
        uint8_t *filled = (uint8_t *)calloc((size_t)tot + 1, 1);
        for (int pass = 2; pass >= 0; pass--) {
            for (int64_t a = 0; a < n_arcs; a++) {
                int32_t g = arc_gate[a];
                int is_cond = arc_cond_pin[a] >= 0;
                int edge = arc_in_edge ? arc_in_edge[a] : 0;
                if (edge < 0 || edge > 2) { set_err(err, errlen, "bad input-edge qualifier"); free(filled); oracle_free(d); return NULL; }
                if (is_cond + (edge != 0) != pass) continue;
                if (g < 0 || g >= G) { set_err(err, errlen, "arc gate out of range"); free(filled); oracle_free(d); return NULL; }
                int32_t k = d->cell_pins[g], j = arc_pin[a];
                if (j < 0 || j >= k) { set_err(err, errlen, "arc pin out of range"); free(filled); oracle_free(d); return NULL; }
                if (arc_rise[a] < 0 || arc_fall[a] < 0) { set_err(err, errlen, "negative delay"); free(filled); oracle_free(d); return NULL; }
                int32_t q = arc_cond_pin[a];
                if (is_cond && (q >= k || q == j)) { set_err(err, errlen, "bad condition pin"); free(filled); oracle_free(d); return NULL; }
                int64_t base = d->dtab_ptr[fanin_ptr[g] + j];
                for (int32_t st = 0; st < (1 << k); st++) {
                    if (is_cond && (((st >> q) & 1) != arc_cond_val[a])) continue;
                    if (edge == 1 && !((st >> j) & 1)) continue;      /* rising input only */
                    if (edge == 2 && ((st >> j) & 1)) continue;       /* falling input only */
                    if (filled[base + 2 * st] > pass + 1) continue;   /* a more specific record holds it */
                    if (filled[base + 2 * st] == pass + 1) {
                        set_err(err, errlen, "two arc records match one pin state"); free(filled); oracle_free(d); return NULL;
                    }
                    filled[base + 2 * st] = (uint8_t)(pass + 1);
                    filled[base + 2 * st + 1] = (uint8_t)(pass + 1);
                    d->dtab[base + 2 * st + 0] = arc_fall[a];
                    d->dtab[base + 2 * st + 1] = arc_rise[a];
                }
            }
        }
        for (int64_t e = 0; e < tot; e++)
            if (!filled[e]) { set_err(err, errlen, "a pin state has no arc record"); free(filled); oracle_free(d); return NULL; }
        free(filled);
    }
    return d;
}

int32_t oracle_level(void *p, int32_t net) { return ((Design *)p)->level[net]; }

/* ---------------------------------------------------------------- heap */
typedef struct {
    Event *pool; int64_t n_pool, cap_pool;
    int64_t *heap; int64_t n_heap, cap_heap;
    int64_t seq;
} Queue;

static int ev_less(const Event *a, const Event *b)
{
    if (a->t != b->t) return a->t < b->t;
    if (a->level != b->level) return a->level < b->level;
    if (a->kind != b->kind) return a->kind < b->kind;
    return a->seq < b->seq;
}

static int64_t push(Queue *q, int64_t t, int32_t level, int32_t kind, int32_t id, int32_t val)
{
    if (q->n_pool == q->cap_pool) {
        q->cap_pool = q->cap_pool ? 2 * q->cap_pool : 1024;
        q->pool = (Event *)realloc(q->pool, sizeof(Event) * (size_t)q->cap_pool);
    }
    if (q->n_heap == q->cap_heap) {
        q->cap_heap = q->cap_heap ? 2 * q->cap_heap : 1024;
        q->heap = (int64_t *)realloc(q->heap, sizeof(int64_t) * (size_t)q->cap_heap);
    }
    int64_t e = q->n_pool++;
    Event *ev = &q->pool[e];
    ev->t = t; ev->level = level; ev->kind = kind; ev->id = id; ev->val = val;
    ev->cancelled = 0; ev->seq = q->seq++;
    int64_t i = q->n_heap++;
    q->heap[i] = e;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (!ev_less(&q->pool[q->heap[i]], &q->pool[q->heap[par]])) break;
        int64_t tmp = q->heap[i]; q->heap[i] = q->heap[par]; q->heap[par] = tmp;
        i = par;
    }
    return e;
}

static int64_t pop(Queue *q)
{
    int64_t top = q->heap[0];
    q->heap[0] = q->heap[--q->n_heap];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < q->n_heap && ev_less(&q->pool[q->heap[l]], &q->pool[q->heap[m]])) m = l;
        if (r < q->n_heap && ev_less(&q->pool[q->heap[r]], &q->pool[q->heap[m]])) m = r;
        if (m == i) break;
        int64_t tmp = q->heap[i]; q->heap[i] = q->heap[m]; q->heap[m] = tmp;
        i = m;
    }
    return top;
}

/* ---------------------------------------------------------------- run */
static int32_t pin_state(const Design *d, const int32_t *pin_val, int32_t g)
{
    int32_t st = 0;
    for (int64_t s = d->fanin_ptr[g]; s < d->fanin_ptr[g + 1]; s++)
        st |= pin_val[s] << (s - d->fanin_ptr[g]);
    return st;
}

/*
 * Simulate cycles [cycle_begin, cycle_end) and ADD per-net TC/T0/T1 into
 * tc/t0/t1 (length n_inputs + n_gates).  Toggle times are absolute, strictly
 * increasing per input.
 *
 * ig (may be NULL) gets the glitch toggles (SAIF's IG; the paper's SAIF
 * output, Section 3, read as follows): in a cycle whose list has L edges,
 * at most one edge is functional (the settled value changes iff L is odd),
 * so the cycle adds L - (L mod 2) glitch toggles.  ig_cycle (may be NULL,
 * length cycle_end - cycle_begin) gets the same toggles summed over all
 * nets per cycle: the cycle-by-cycle glitch profile whose peaks are the
 * hot spots the glitch-optimization flow of Section 4 looks for.
 *
 * late_cycle (may be NULL, length cycle_end - cycle_begin) counts, per
 * cycle, the nets whose last edge in the cycle, or that edge's arrival at
 * one of the net's fanout pins through the pin's wire delay (rise or fall
 * by the value after the edge), lies at or after the period T.  A cycle
 * whose count is 0 ends quiescent: every net holds the zero-delay value of
 * the inputs and nothing is pending, so the next cycle's isolated start
 * (the settled values) is exactly the state a continuous run would reach.
 * The test is conservative: such an arrival may still be filtered.
 *
 * Probes: for probe p, if cycle_begin <= probe_cycle[p] < cycle_end, the
 * initial value, edge count and up to probe_cap edge times of net
 * probe_net[p] in that cycle are written to probe_init[p], probe_len[p] and
 * probe_times[p*probe_cap ...].
 *
 * stats[0] += processed (non-cancelled) events, stats[1] += recorded edges.
 * net_filter: 1 = the interconnect inertial filter, 0 = transport wire
 * delays (the feature study's "no net delay" filtering).
 * Returns 0, or -1 on an internal inconsistency.
 */
int32_t oracle_run(void *p, int32_t period, int32_t n_cycles,
                   const uint8_t *init, const int64_t *toggle_ptr, const int64_t *toggle_ps,
                   int32_t cycle_begin, int32_t cycle_end,
                   int64_t *tc, int64_t *t0, int64_t *t1, int64_t *ig, int64_t *ig_cycle,
                   int64_t *late_cycle, int32_t n_probe, const int32_t *probe_net, const int32_t *probe_cycle,
                   int32_t *probe_init, int32_t *probe_len, int32_t *probe_times, int32_t probe_cap,
                   int64_t *stats, int32_t net_filter)
{
    Design *d = (Design *)p;
    int32_t I = d->n_inputs, G = d->n_gates, N = d->n_nets;
    int64_t F = d->fanin_ptr[G];
    const int64_t T = period;
    (void)n_cycles;

    int32_t *net_val = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    int32_t *start_val = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    int32_t *pin_val = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F + 1));
    int64_t *arc_pend = (int64_t *)malloc(sizeof(int64_t) * (size_t)(F + 1));
    int64_t *arc_pend_t = (int64_t *)malloc(sizeof(int64_t) * (size_t)(F + 1));
    int64_t *gate_pend = (int64_t *)malloc(sizeof(int64_t) * (size_t)(G + 1));
    int64_t *eval_t = (int64_t *)malloc(sizeof(int64_t) * (size_t)(G + 1));
    int32_t *sw_mask = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G + 1));
    int64_t *tcur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(I + 1));
    /* edges recorded during a cycle, in processing (= time) order */
    int64_t n_rec = 0, cap_rec = 1024;
    int32_t *rec_net = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap_rec);
    int64_t *rec_t = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap_rec);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    int64_t *ord = NULL; int64_t cap_ord = 0;
    Queue q; memset(&q, 0, sizeof(q));
    int32_t rc = 0;

    /* first toggle of each input at or after cycle_begin*T */
    for (int32_t i = 0; i < I; i++) {
        int64_t k = toggle_ptr[i];
        while (k < toggle_ptr[i + 1] && toggle_ps[k] < (int64_t)cycle_begin * T) k++;
        tcur[i] = k;
    }

    for (int32_t c = cycle_begin; c < cycle_end && rc == 0; c++) {
        int64_t c0 = (int64_t)c * T;
        /* inputs: value just before c*T */
        for (int32_t i = 0; i < I; i++)
            net_val[i] = (init[i] ^ (int32_t)((tcur[i] - toggle_ptr[i]) & 1)) & 1;
        /* zero-delay settle in level order */
        for (int32_t x = 0; x < G; x++) {
            int32_t g = d->topo[x], st = 0;
            for (int64_t s = d->fanin_ptr[g]; s < d->fanin_ptr[g + 1]; s++)
                st |= net_val[d->fanin_net[s]] << (s - d->fanin_ptr[g]);
            net_val[I + g] = (int32_t)((d->truth[g] >> st) & 1);
        }
        for (int64_t s = 0; s < F; s++) { pin_val[s] = net_val[d->fanin_net[s]]; arc_pend[s] = -1; }
        for (int32_t g = 0; g < G; g++) { gate_pend[g] = -1; eval_t[g] = -1; sw_mask[g] = 0; }
        memcpy(start_val, net_val, sizeof(int32_t) * (size_t)N);

        q.n_pool = 0; q.n_heap = 0; q.seq = 0;
        for (int32_t i = 0; i < I; i++) {
            int64_t k = tcur[i];
            while (k < toggle_ptr[i + 1] && toggle_ps[k] < c0 + T) {
                /* input edges alternate; the value is set when the edge is applied */
                push(&q, toggle_ps[k] - c0, 0, EV_NET, i, -1);
                k++;
            }
            tcur[i] = k;
        }
        n_rec = 0;

        while (q.n_heap > 0) {
            int64_t e = pop(&q);
            Event ev = q.pool[e];
            if (ev.cancelled) continue;
            if (stats) stats[0]++;
            if (ev.kind == EV_NET) {
                int32_t n = ev.id;
                int32_t v = (ev.val < 0) ? (net_val[n] ^ 1) : ev.val;
                if (v == net_val[n]) { rc = -1; break; }
                if (n >= I) gate_pend[n - I] = -1;
                net_val[n] = v;
                if (n_rec == cap_rec) {
                    cap_rec *= 2;
                    rec_net = (int32_t *)realloc(rec_net, sizeof(int32_t) * (size_t)cap_rec);
                    rec_t = (int64_t *)realloc(rec_t, sizeof(int64_t) * (size_t)cap_rec);
                }
                rec_net[n_rec] = n; rec_t[n_rec] = ev.t; n_rec++;
                for (int64_t f = d->fo_ptr[n]; f < d->fo_ptr[n + 1]; f++) {
                    int32_t s = d->fo_slot[f];
                    int32_t g = d->slot_gate[s];
                    int64_t delta = v ? d->wire_r[s] : d->wire_f[s];
                    /* inertial: the net edge comes before the pending pin
                     * edge matures; transport: the new arrival is no later
                     * than the last scheduled, still pending one */
                    int32_t cancel = arc_pend[s] >= 0 &&
                                     (net_filter ? ev.t < arc_pend_t[s] : ev.t + delta <= arc_pend_t[s]);
                    if (cancel) {
                        q.pool[arc_pend[s]].cancelled = 1;      /* the pulse vanishes */
                        arc_pend[s] = -1;
                    } else {
                        int64_t pe = push(&q, ev.t + delta, d->level[I + g], EV_PIN, s, v);
                        arc_pend[s] = pe;
                        arc_pend_t[s] = ev.t + delta;
                    }
                }
            } else if (ev.kind == EV_PIN) {
                int32_t s = ev.id;
                if (arc_pend[s] == e) arc_pend[s] = -1;
                if (pin_val[s] == ev.val) { rc = -1; break; }
                pin_val[s] = ev.val;
                int32_t g = d->slot_gate[s];
                sw_mask[g] |= 1 << d->slot_pin[s];
                if (eval_t[g] != ev.t) {
                    eval_t[g] = ev.t;
                    push(&q, ev.t, d->level[I + g], EV_EVAL, g, 0);
                }
            } else {
                int32_t g = ev.id;
                int32_t st = pin_state(d, pin_val, g);
                int32_t y = (int32_t)((d->truth[g] >> st) & 1);
                int32_t cur = net_val[I + g];
                int32_t pending = gate_pend[g] >= 0;
                int32_t z = pending ? (cur ^ 1) : cur;
                if (y != z) {
                    if (pending) {
                        if (q.pool[gate_pend[g]].t <= ev.t) { rc = -1; break; }
                        q.pool[gate_pend[g]].cancelled = 1;   /* output pulse narrower than its delay */
                        gate_pend[g] = -1;
                    } else {
                        int64_t dl = -1;
                        for (int64_t s = d->fanin_ptr[g]; s < d->fanin_ptr[g + 1]; s++) {
                            if (!((sw_mask[g] >> (s - d->fanin_ptr[g])) & 1)) continue;
                            int64_t x = d->dtab[d->dtab_ptr[s] + 2 * st + y];
                            if (dl < 0 || x < dl) dl = x;
                        }
                        gate_pend[g] = push(&q, ev.t + dl, d->level[I + g], EV_NET, I + g, y);
                    }
                }
                sw_mask[g] = 0;
            }
        }
        if (rc) break;
        if (stats) stats[1] += n_rec;

        /* group recorded edges by net (stable: keeps time order) */
        if (cap_ord < n_rec + 1) {
            cap_ord = n_rec + 1;
            ord = (int64_t *)realloc(ord, sizeof(int64_t) * (size_t)cap_ord);
        }
        memset(cnt, 0, sizeof(int64_t) * (size_t)(N + 1));
        for (int64_t r = 0; r < n_rec; r++) cnt[rec_net[r] + 1]++;
        for (int32_t n = 0; n < N; n++) cnt[n + 1] += cnt[n];
        {
            int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
            memcpy(fill, cnt, sizeof(int64_t) * (size_t)(N + 1));
            for (int64_t r = 0; r < n_rec; r++) ord[fill[rec_net[r]]++] = r;
            free(fill);
        }
        for (int32_t n = 0; n < N; n++) {
            int64_t a = cnt[n], b = cnt[n + 1];
            tc[n] += b - a;
            if (ig) ig[n] += (b - a) - ((b - a) & 1);
            if (ig_cycle) ig_cycle[c - cycle_begin] += (b - a) - ((b - a) & 1);
            if (late_cycle && b > a) {
                int64_t last = rec_t[ord[b - 1]], reach = last;
                int32_t v_end = start_val[n] ^ (int32_t)((b - a) & 1);
                for (int64_t k = d->fo_ptr[n]; k < d->fo_ptr[n + 1]; k++) {
                    int32_t s = d->fo_slot[k];
                    int64_t r = last + (v_end ? d->wire_r[s] : d->wire_f[s]);
                    if (r > reach) reach = r;
                }
                if (reach >= T) late_cycle[c - cycle_begin]++;
            }
            /* time at 1 and time at 0 in [0, T), summed segment by segment */
            int32_t v = start_val[n];
            int64_t prev = 0, on = 0, off = 0;
            for (int64_t r = a; r <= b; r++) {
                int64_t end = (r < b) ? rec_t[ord[r]] : T;
                if (r < b && r > a && rec_t[ord[r]] <= rec_t[ord[r - 1]]) { rc = -1; }
                int64_t lo = prev < T ? prev : T, hi = end < T ? end : T;
                if (hi > lo) { if (v) on += hi - lo; else off += hi - lo; }
                v ^= 1;
                prev = end;
            }
            t1[n] += on;
            t0[n] += off;
        }
        for (int32_t pp = 0; pp < n_probe; pp++) {
            if (probe_cycle[pp] != c) continue;
            int32_t n = probe_net[pp];
            int64_t a = cnt[n], b = cnt[n + 1];
            probe_init[pp] = start_val[n];
            probe_len[pp] = (int32_t)(b - a);
            for (int64_t r = a; r < b && r - a < probe_cap; r++)
                probe_times[(int64_t)pp * probe_cap + (r - a)] = (int32_t)rec_t[ord[r]];
        }
    }

    free(net_val); free(start_val); free(pin_val); free(arc_pend); free(arc_pend_t);
    free(gate_pend); free(eval_t); free(sw_mask); free(tcur); free(rec_net); free(rec_t);
    free(cnt); free(ord); free(q.pool); free(q.heap);
    return rc;
}
