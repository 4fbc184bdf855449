// gfx950 kernels of the gate-level re-simulator.
//
// Work decomposition (GATSPI Section 3: design parallelism within a logic
// level, cycle parallelism across the known-stimulus cycles): one 64-lane
// wavefront evaluates one gate over one tile of 64 consecutive cycles, one
// lane per cycle.  Waveform data of a (net, tile) is one contiguous chunk, so
// the 64 lanes of a wave read neighbouring words of the same chunk.
#include "internal.h"

namespace gs {

// --------------------------------------------------------------------------
// wave-level helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kLanes; d <<= 1) {
        uint32_t o = __shfl_up(v, d, kLanes);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ int32_t wave_sum(int32_t v)
{
#pragma unroll
    for (int d = kLanes / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kLanes);
    return v;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Places a wave's finished chunk: one atomic bump of the transition arena
// for the whole wave, then lane ends and the chunk header.  Returns false
// (and writes an empty, in-bounds chunk) when the arena is full or the chunk
// exceeds 16-bit lane ends; the host then redoes the window.
__device__ __forceinline__ bool place_chunk(const WinView &win, uint64_t ci, uint32_t incl, uint32_t total,
                                            uint64_t mask, int lane, uint32_t salt, uint64_t &base)
{
    bool ok = true;
    if (total > kMaxChunk) {
        if (lane == 0) atomicOr(&win.flags[1], 1u);
        ok = false;
    }
    uint64_t b = 0;
    if (ok && total > 0) {
        const uint32_t stripe = (blockIdx.x + salt) & win.stripe_mask;
        if (lane == 0) b = atomicAdd(win.bump + (size_t)stripe * kBumpStride, (unsigned long long)total);
        b = uniform64(b);
        if (b + total > win.slice_words) {
            if (lane == 0) atomicOr(&win.flags[0], 1u);
            ok = false;
        }
        b += (uint64_t)stripe * win.slice_words;
    }
    win.ends[ci * kLanes + lane] = ok ? (uint16_t)incl : (uint16_t)0;
    if (lane == 0) {
        ChunkHdr h;
        h.off = ok ? b : 0;
        h.mask = mask;
        win.hdr[ci] = h;
    }
    base = b;
    return ok;
}

// --------------------------------------------------------------------------
// small utility kernels (also used instead of memset so that every launch
// sequence can be captured into a graph)
// --------------------------------------------------------------------------
__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n, unsigned long long v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(unsigned int *p, uint64_t n, unsigned int v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void add_u64_kernel(unsigned long long *dst, const unsigned long long *src, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] += src[i];
}

static unsigned grid_for(uint64_t n)
{
    uint64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b == 0) b = 1;
    return (unsigned)b;
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int *p, uint64_t n, unsigned int v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_add_u64(unsigned long long *dst, const unsigned long long *src, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(add_u64_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Levelizer (Section 3: the netlist is partitioned by logic level).  Level 0
// holds the inputs; a gate's level is 1 + the largest level of its fanin
// nets.  Relaxation sweeps: a gate takes its level once every fanin has
// one; a sweep that places nothing while gates remain proves a cycle.
// counters[0] = gates placed in the sweep, counters[1] = gates still open.
// --------------------------------------------------------------------------
__global__ void level_init_kernel(int32_t *level, int32_t n_inputs, int32_t n_nets)
{
    int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < n_nets) level[n] = n < n_inputs ? 0 : -1;
}

__global__ void level_step_kernel(const int64_t *__restrict__ fanin_ptr, const int32_t *__restrict__ fanin_net,
                                  int32_t *level, int32_t n_inputs, int32_t n_gates, unsigned int *counters)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gates) return;
    if (level[n_inputs + g] >= 0) return;
    int32_t mx = 0;
    for (int64_t s = fanin_ptr[g]; s < fanin_ptr[g + 1]; s++) {
        int32_t l = __hip_atomic_load(&level[fanin_net[s]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (l < 0) {
            atomicAdd(&counters[1], 1u);
            return;
        }
        mx = l > mx ? l : mx;
    }
    __hip_atomic_store(&level[n_inputs + g], mx + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicAdd(&counters[0], 1u);
}

// count_only: cursor[level] += 1 per gate (histogram).  Otherwise cursor
// holds each level's first position and gates are scattered into perm.
__global__ void level_bucket_kernel(const int32_t *__restrict__ level, int32_t n_inputs, int32_t n_gates,
                                    unsigned int *cursor, int32_t *perm, int count_only)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gates) return;
    int32_t l = level[n_inputs + g];
    unsigned int pos = atomicAdd(&cursor[l], 1u);
    if (!count_only) perm[pos] = g;
}

hipError_t launch_level_init(int32_t *level, int32_t n_inputs, int32_t n_gates, hipStream_t s)
{
    int32_t n = n_inputs + n_gates;
    hipLaunchKernelGGL(level_init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, level, n_inputs, n);
    return hipGetLastError();
}

hipError_t launch_level_step(const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t *level,
                             int32_t n_inputs, int32_t n_gates, unsigned int *counters, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(level_step_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, fanin_ptr, fanin_net,
                       level, n_inputs, n_gates, counters);
    return hipGetLastError();
}

hipError_t launch_level_bucket(const int32_t *level, int32_t n_inputs, int32_t n_gates, unsigned int *cursor,
                               int32_t *perm, int count_only, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(level_bucket_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, level, n_inputs,
                       n_gates, cursor, perm, count_only);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Stimulus expansion (the input restructuring GATSPI does before its
// kernels, Section 4): absolute toggle times of input i become the
// (input, tile) chunks of the window, in cycle-local time, with the
// pre-cycle value of every cycle in the chunk mask.  Also adds the inputs'
// SAIF counts.
// --------------------------------------------------------------------------
__device__ __forceinline__ int64_t lower_bound64(const int64_t *__restrict__ a, int64_t lo, int64_t hi, int64_t key)
{
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void expand_kernel(StimView st, WinView win, SaifAcc acc, int32_t cycle0,
                                                     uint32_t salt, uint64_t n_waves)
{
    const int lane = threadIdx.x & (kLanes - 1);
    const uint32_t wib = uniform(threadIdx.x / kLanes);
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / kLanes) + wib;
    if (w >= n_waves) return;
    const uint32_t ntile = (uint32_t)win.n_tiles;
    const uint32_t i = uniform((uint32_t)(w / ntile));
    const uint32_t tile = uniform((uint32_t)(w % ntile));
    const int32_t lc = (int32_t)(tile * kLanes + lane);
    const bool active = lc < win.n_cycles;
    const int64_t T = st.period;
    const int64_t c0 = (int64_t)(cycle0 + lc) * T;
    const int64_t lo = st.toggle_ptr[i], hi = st.toggle_ptr[i + 1];
    int64_t s = 0, e = 0;
    if (active) {
        s = lower_bound64(st.toggle_ps, lo, hi, c0);
        e = lower_bound64(st.toggle_ps, s, hi, c0 + T);
    }
    const uint32_t cnt = (uint32_t)(e - s);
    const int v0 = active ? (int)((st.init[i] + (uint64_t)(s - lo)) & 1) : 0;
    const uint32_t incl = wave_incl_scan(cnt, lane);
    const uint32_t total = uniform(__shfl(incl, kLanes - 1, kLanes));
    const uint64_t mask = __ballot(v0 != 0);
    const uint64_t ci = (uint64_t)i * ntile + tile;
    uint64_t base;
    const bool ok = place_chunk(win, ci, incl, total, mask, lane, salt, base);
    // time at 1 inside [0, T): final value * T - sum of rising-edge times + sum of falling-edge times
    int v = v0, a = 0;
    for (uint32_t j = 0; j < cnt; j++) {
        int32_t tl = (int32_t)(st.toggle_ps[s + j] - c0);
        if (ok) win.times[base + (incl - cnt) + j] = tl;
        v ^= 1;
        a += v ? -tl : tl;
    }
    const int32_t t1 = active ? v * (int32_t)T + a : 0;
    const int32_t sum1 = wave_sum(t1);
    const uint32_t nact = (uint32_t)__popcll(__ballot(active));
    if (lane == 0) {
        atomicAdd(&acc.tc[i], (unsigned long long)total);
        atomicAdd(&acc.t1[i], (unsigned long long)(int64_t)sum1);
        atomicAdd(&acc.t0[i], (unsigned long long)((int64_t)nact * T - sum1));
    }
}

hipError_t launch_expand(StimView st, WinView win, SaifAcc acc, int32_t cycle0, uint32_t salt, hipStream_t s)
{
    uint64_t n_waves = (uint64_t)st.n_inputs * (uint64_t)win.n_tiles;
    if (n_waves == 0) return hipSuccess;
    const int wpb = 4;
    uint64_t blocks = (n_waves + wpb - 1) / wpb;
    hipLaunchKernelGGL(expand_kernel, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, st, win, acc, cycle0, salt,
                       n_waves);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Gate evaluation (Algorithm 1, one lane per (gate, cycle)).
//
// Per lane: the fanin pins' cycle-local transition lists are walked in time
// order.  At each earliest arrival time t every pin arriving at t switches
// (MSI resolution), the truth table gives the new value y, and when y
// differs from the value the output is heading to, the gate inertial filter
// either cancels the pending output edge (t earlier than it) or appends a
// new edge at t + delay, delay = smallest arc delay of the switching pins in
// the post-switch pin state.  With interconnect delays, each pin's arrivals
// come from its net's edges through the wire inertial filter (a net pulse
// narrower than the wire delay of its leading edge is skipped).
//
// Output edges are staged in LDS (CAP per lane, lane-interleaved so that
// every store is bank-conflict free), the wave prefix-sums the lane counts,
// reserves its chunk with one atomic, and copies out.  Lanes whose list
// outgrew CAP run the same walk again, writing straight to their reserved
// place in global memory.  SAIF counts of the output net are reduced over
// the wave and added with one atomic each.
// --------------------------------------------------------------------------
template <int K, bool WIRES>
struct Lane {
    const int32_t *chunk[K];
    uint32_t idx[K], end[K];
    int32_t a[K];
    int32_t q[K], r0[K], f0[K], r1[K], f1[K], wr[K], wf[K];
    uint32_t state;

    __device__ __forceinline__ void advance(int j)
    {
        if (!WIRES) {
            a[j] = idx[j] < end[j] ? chunk[j][idx[j]] : kInf;
            return;
        }
        const int pv = (state >> j) & 1;
        for (;;) {
            if (idx[j] >= end[j]) {
                a[j] = kInf;
                return;
            }
            const int32_t e0 = chunk[j][idx[j]];
            const int32_t d = pv ? wf[j] : wr[j];       // the net edge goes to !pv
            if (idx[j] + 1 < end[j] && chunk[j][idx[j] + 1] - e0 < d) {
                idx[j] += 2;                            // pulse narrower than the wire delay
                continue;
            }
            a[j] = e0 + d;
            return;
        }
    }
};

// MODE 0: stage into LDS (at most CAP entries per lane).  MODE 1: write to
// global memory at dst[0 .. keep) (entries at or beyond `keep` are retracted
// before the walk ends, so they are not stored).
template <int K, bool WIRES, int MODE, int CAP>
__device__ __forceinline__ void walk(Lane<K, WIRES> &L, uint64_t truth, int32_t T, int z, int32_t *lds_lane,
                                     int32_t *dst, int32_t keep, int32_t &cnt_out, int32_t &acc_out, int32_t &z_out)
{
#pragma unroll
    for (int j = 0; j < K; j++) L.advance(j);
    int32_t W = 0, Wp = 0, cnt = 0, acc = 0;
    for (;;) {
        int32_t t = L.a[0];
#pragma unroll
        for (int j = 1; j < K; j++) t = min(t, L.a[j]);
        if (t == kInf) break;
        uint32_t sw = 0;
#pragma unroll
        for (int j = 0; j < K; j++) {
            if (L.a[j] == t) {
                sw |= 1u << j;
                L.state ^= 1u << j;
                L.idx[j]++;
                L.advance(j);
            }
        }
        const int y = (int)((truth >> L.state) & 1);
        if (y != z) {
            int32_t d = kInf;
#pragma unroll
            for (int j = 0; j < K; j++) {
                // arithmetic selects: a select between array elements would
                // become an address select and force the arrays to scratch
                const int32_t sel = -(int32_t)((L.state >> L.q[j]) & 1);
                const int32_t rise = L.r0[j] + (sel & (L.r1[j] - L.r0[j]));
                const int32_t fall = L.f0[j] + (sel & (L.f1[j] - L.f0[j]));
                const int32_t dj = fall + ((-y) & (rise - fall));
                const int32_t m = -(int32_t)((sw >> j) & 1);      // pin j switched at t
                d = min(d, (dj & m) | (kInf & ~m));
            }
            const bool retract = t < W;
            const int32_t e = retract ? W : t + d;
            const int32_t ce = min(e, T);
            acc += y ? -ce : ce;
            if (retract) {
                cnt--;
                W = Wp;
            } else {
                if (MODE == 0) {
                    if (cnt < CAP) lds_lane[cnt * kLanes] = t + d;
                } else {
                    if (cnt < keep) dst[cnt] = t + d;
                }
                cnt++;
                Wp = W;
                W = t + d;
            }
            z = y;
        }
    }
    cnt_out = cnt;
    acc_out = acc;
    z_out = z;
}

template <int K, bool WIRES, int CAP>
__device__ __forceinline__ void eval_gate(const Seg &sg, const GateRec &g, uint32_t tile, int lane, int32_t *lds)
{
    const WinView &win = sg.win;
    const int32_t lc = (int32_t)(tile * kLanes) + lane;
    const bool active = lc < win.n_cycles;
    const int32_t T = win.period;
    Lane<K, WIRES> L;
    uint32_t idx0[K];
    L.state = 0;
#pragma unroll
    for (int j = 0; j < K; j++) {
        const PinRec pr = sg.pins[g.pin0 + j];
        const uint64_t ci = (uint64_t)(uint32_t)pr.net * (uint32_t)win.n_tiles + tile;
        const ChunkHdr h = win.hdr[ci];
        const uint16_t *e = win.ends + ci * kLanes;
        const uint32_t hi = e[lane];
        const uint32_t lo = lane > 0 ? e[lane - 1] : 0u;
        L.chunk[j] = win.times + h.off;
        L.idx[j] = active ? lo : 0u;
        L.end[j] = active ? hi : 0u;
        idx0[j] = L.idx[j];
        L.state |= (uint32_t)((h.mask >> lane) & 1) << j;
        L.q[j] = pr.q;
        L.r0[j] = pr.r0;
        L.f0[j] = pr.f0;
        L.r1[j] = pr.r1;
        L.f1[j] = pr.f1;
        L.wr[j] = pr.wr;
        L.wf[j] = pr.wf;
    }
    const uint32_t state0 = L.state;
    const int y0 = (int)((g.truth >> state0) & 1);     // zero-delay settled value at t = 0

    int32_t cnt, acc, z;
    walk<K, WIRES, 0, CAP>(L, g.truth, T, y0, lds + lane, nullptr, 0, cnt, acc, z);

    const uint32_t ucnt = (uint32_t)cnt;
    const uint32_t incl = wave_incl_scan(ucnt, lane);
    const uint32_t total = uniform(__shfl(incl, kLanes - 1, kLanes));
    const uint64_t mask = __ballot(active && y0);
    const uint64_t ci = (uint64_t)g.out * (uint32_t)win.n_tiles + tile;
    uint64_t base;
    const bool ok = place_chunk(win, ci, incl, total, mask, lane, sg.salt, base);
    const uint32_t excl = incl - ucnt;
    if (ok) {
        int32_t *out = win.times + base + excl;
        const int32_t n = cnt < CAP ? cnt : CAP;
        for (int32_t i = 0; i < n; i++) out[i] = lds[lane + i * kLanes];
        const uint64_t spill = __ballot(cnt > CAP);
        if (spill) {
            if (cnt > CAP) {
#pragma unroll
                for (int j = 0; j < K; j++) L.idx[j] = idx0[j];
                L.state = state0;
                int32_t c2, a2, z2;
                walk<K, WIRES, 1, CAP>(L, g.truth, T, y0, nullptr, out, cnt, c2, a2, z2);
            }
            if (lane == 0) atomicAdd(&win.flags[2], (unsigned int)__popcll(spill));
        }
    }
    const int32_t t1 = active ? z * T + acc : 0;
    const int32_t sum1 = wave_sum(t1);
    const uint32_t nact = (uint32_t)__popcll(__ballot(active));
    if (lane == 0) {
        atomicAdd(&sg.saif.tc[g.out], (unsigned long long)total);
        atomicAdd(&sg.saif.t1[g.out], (unsigned long long)(int64_t)sum1);
        atomicAdd(&sg.saif.t0[g.out], (unsigned long long)((int64_t)nact * T - sum1));
    }
}

__device__ __forceinline__ int find_seg(const Seg *__restrict__ segs, int n, uint64_t w)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].wave_begin <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <bool WIRES, int CAP, int KMAX>
__global__ __launch_bounds__(512) void gate_eval_kernel(const Seg *__restrict__ segs, int32_t n_segs, uint64_t n_waves)
{
    extern __shared__ int32_t lds_all[];
    const int lane = threadIdx.x & (kLanes - 1);
    const uint32_t wpb = blockDim.x / kLanes;
    const uint32_t wib = uniform(threadIdx.x / kLanes);
    const uint64_t w = (uint64_t)blockIdx.x * wpb + wib;
    if (w >= n_waves) return;
    const int si = n_segs == 1 ? 0 : find_seg(segs, n_segs, w);
    const Seg &sg = segs[si];
    const uint32_t local = (uint32_t)(w - sg.wave_begin);
    const uint32_t ntile = (uint32_t)sg.win.n_tiles;
    const uint32_t gi = local / ntile;
    const uint32_t tile = local - gi * ntile;
    const GateRec g = sg.gates[sg.gate_begin + gi];
    int32_t *lds = lds_all + (size_t)wib * CAP * kLanes;
    switch (g.k) {
    case 1: eval_gate<1, WIRES, CAP>(sg, g, tile, lane, lds); break;
    case 2: eval_gate<2, WIRES, CAP>(sg, g, tile, lane, lds); break;
    case 3: eval_gate<3, WIRES, CAP>(sg, g, tile, lane, lds); break;
    case 4: if (KMAX >= 4) eval_gate<(KMAX >= 4 ? 4 : 1), WIRES, CAP>(sg, g, tile, lane, lds); break;
    case 5: if (KMAX >= 5) eval_gate<(KMAX >= 5 ? 5 : 1), WIRES, CAP>(sg, g, tile, lane, lds); break;
    case 6: if (KMAX >= 6) eval_gate<(KMAX >= 6 ? 6 : 1), WIRES, CAP>(sg, g, tile, lane, lds); break;
    default: break;
    }
}

template <bool WIRES, int KMAX>
static hipError_t launch_ge(const Seg *segs, int32_t n_segs, uint64_t n_waves, int32_t cap, int32_t wpb, hipStream_t s)
{
    const uint64_t blocks = (n_waves + wpb - 1) / wpb;
    const size_t lds = (size_t)wpb * cap * kLanes * sizeof(int32_t);
    const dim3 grid((unsigned)blocks), block(kLanes * wpb);
    switch (cap) {
    case 4: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 4, KMAX>), grid, block, lds, s, segs, n_segs, n_waves); break;
    case 8: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 8, KMAX>), grid, block, lds, s, segs, n_segs, n_waves); break;
    case 16: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 16, KMAX>), grid, block, lds, s, segs, n_segs, n_waves); break;
    case 32: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 32, KMAX>), grid, block, lds, s, segs, n_segs, n_waves); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gate_eval(const Seg *segs, int32_t n_segs, uint64_t n_waves, int32_t wires, int32_t cap,
                            int32_t wpb, int32_t kmax, hipStream_t s)
{
    if (n_waves == 0) return hipSuccess;
    if (wpb < 1 || wpb > 8) return hipErrorInvalidValue;
    if (kmax <= 3)
        return wires ? launch_ge<true, 3>(segs, n_segs, n_waves, cap, wpb, s)
                     : launch_ge<false, 3>(segs, n_segs, n_waves, cap, wpb, s);
    return wires ? launch_ge<true, 6>(segs, n_segs, n_waves, cap, wpb, s)
                 : launch_ge<false, 6>(segs, n_segs, n_waves, cap, wpb, s);
}

}  // namespace gs
