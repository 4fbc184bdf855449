// gfx950 kernels of the gate-level re-simulator.
//
// Work decomposition (GATSPI Section 3: design parallelism within a logic
// level, cycle parallelism across the known-stimulus cycles): one 64-lane
// wavefront evaluates one gate over one tile of 64 consecutive cycles, one
// lane per cycle.  Waveform data of a (net, tile) is one contiguous chunk, so
// the 64 lanes of a wave read neighbouring words of the same chunk.
#include "internal.h"

#include <mutex>

namespace gs {

// --------------------------------------------------------------------------
// Static device scratch of the allocation-free simulate call: one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel (on the host it names a stand-in, not device memory); it uses
// the per-device address that scratch_region looks up once per device.
// --------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_region(int device, void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current first
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

// Explicit global address space: pointers read out of the segment table
// would otherwise stay generic and every access would become a flat
// instruction that waits on both the vector-memory and the LDS counters.
#if defined(__HIP_DEVICE_COMPILE__)
#define GAS __attribute__((address_space(1)))
#else
#define GAS
#endif

template <typename T>
__device__ __forceinline__ GAS T *glob(T *p)
{
    return (GAS T *)p;
}

// Read-only view for wave-uniform data that the current launch never
// writes (gate and pin records, and chunk headers of lower levels, written
// by earlier launches): uniform addresses then load through the scalar
// cache with s_load.
#if defined(__HIP_DEVICE_COMPILE__)
#define CAS __attribute__((address_space(4)))
#else
#define CAS
#endif

template <typename T>
__device__ __forceinline__ const CAS T *kons(const T *p)
{
    return (const CAS T *)p;
}



// --------------------------------------------------------------------------
// wave-level helpers
// --------------------------------------------------------------------------
// Cross-lane data movement through DPP (no LDS round trip).  row_shr:n
// shifts within each row of 16 lanes; row_bcast:15 / row_bcast:31 carry the
// last lane of a row into the following rows.  Lanes without a source
// (and rows masked off) receive 0.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp0(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, BANK_MASK, true);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    x += dpp0<0x111>(x);             // row_shr:1
    x += dpp0<0x112>(x);             // row_shr:2
    x += dpp0<0x114>(x);             // row_shr:4
    x += dpp0<0x118>(x);             // row_shr:8
    x += dpp0<0x142, 0xa>(x);        // row_bcast:15 into rows 1 and 3
    x += dpp0<0x143, 0xc>(x);        // row_bcast:31 into rows 2 and 3
    return x;
}

// Sum of a 64-bit value over the 64 lanes (every lane gets it): the
// inclusive scan on both halves, carrying the low half's overflow.
__device__ __forceinline__ int64_t wave_sum64(int64_t x)
{
    uint64_t v = (uint64_t)x;
#define GS_SCAN64_STEP(CTRL, RM)                                                                     \
    {                                                                                                \
        const uint32_t lo = dpp0<CTRL, RM>((uint32_t)v), hi = dpp0<CTRL, RM>((uint32_t)(v >> 32)); \
        v += ((uint64_t)hi << 32) | lo;                                                              \
    }
    GS_SCAN64_STEP(0x111, 0xf)
    GS_SCAN64_STEP(0x112, 0xf)
    GS_SCAN64_STEP(0x114, 0xf)
    GS_SCAN64_STEP(0x118, 0xf)
    GS_SCAN64_STEP(0x142, 0xa)
    GS_SCAN64_STEP(0x143, 0xc)
#undef GS_SCAN64_STEP
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, kLanes - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), kLanes - 1);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Value of lane-1 in every lane (0 in lane 0): wave_shr:1.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x)
{
    return dpp0<0x138>(x);
}

__device__ __forceinline__ int32_t lane63(uint32_t x)
{
    return __builtin_amdgcn_readlane((int)x, kLanes - 1);
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

// dst += src unless a window flag (arena full / chunk overflow) is set.
__global__ void add_u64_guarded_kernel(unsigned long long *dst, const unsigned long long *src, uint64_t n,
                                       const unsigned int *flags)
{
    if (flags[0] | flags[1] | flags[3]) return;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] += src[i];
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

hipError_t launch_add_u64_guarded(unsigned long long *dst, const unsigned long long *src, uint64_t n,
                                  const unsigned int *flags, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(add_u64_guarded_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n, flags);
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
// nets.  Frontier order: every gate counts its fanins driven by gates
// (`pending`) and every gate output lists its sink gates (a fanout CSR);
// the gates without such fanins form level 1, and a frontier's gates
// release their sinks, a sink joining the next frontier when its last fanin
// gate has been placed (its level computed then from its fanins' levels).
// The work is one pass over the fanins; gates never placed sit on a cycle.
// --------------------------------------------------------------------------
__global__ void level_init_kernel(int32_t *level, int32_t n_inputs, int32_t n_nets)
{
    int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < n_nets) level[n] = n < n_inputs ? 0 : -1;
}

// pending[g] = fanins of g driven by gates; fo_cnt[h] += 1 for every such
// fanin h (a gate output), the size of h's sink list.
__global__ void fanout_count_kernel(const int64_t *__restrict__ fanin_ptr, const int32_t *__restrict__ fanin_net,
                                    int32_t n_inputs, int32_t n_gates, unsigned int *pending, unsigned int *fo_cnt)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gates) return;
    unsigned int c = 0;
    for (int64_t s = fanin_ptr[g]; s < fanin_ptr[g + 1]; s++) {
        const int32_t n = fanin_net[s];
        if (n >= n_inputs) {
            atomicAdd(&fo_cnt[n - n_inputs], 1u);
            c++;
        }
    }
    pending[g] = c;
}

// Sink lists: fo[fo_ptr[h] ...] = the gates reading gate h's output.
__global__ void fanout_fill_kernel(const int64_t *__restrict__ fanin_ptr, const int32_t *__restrict__ fanin_net,
                                   int32_t n_inputs, int32_t n_gates, const int64_t *__restrict__ fo_ptr,
                                   unsigned int *cursor, int32_t *fo)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gates) return;
    for (int64_t s = fanin_ptr[g]; s < fanin_ptr[g + 1]; s++) {
        const int32_t n = fanin_net[s];
        if (n >= n_inputs) {
            const unsigned int k = atomicAdd(&cursor[n - n_inputs], 1u);
            fo[fo_ptr[n - n_inputs] + k] = g;
        }
    }
}

// The first frontier: gates fed by inputs only, at level 1.
__global__ void level_seed_kernel(const unsigned int *__restrict__ pending, int32_t *level, int32_t n_inputs,
                                  int32_t n_gates, int32_t *frontier, unsigned int *size)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gates || pending[g] != 0) return;
    level[n_inputs + g] = 1;
    frontier[atomicAdd(size, 1u)] = g;
}

// One frontier: each of its gates releases its sinks; the sink whose last
// gate fanin this is takes 1 + the largest level of its fanins (all placed
// by now) and joins the next frontier.
__global__ void level_frontier_kernel(const int32_t *__restrict__ frontier, unsigned int n,
                                      const int64_t *__restrict__ fo_ptr, const int32_t *__restrict__ fo,
                                      const int64_t *__restrict__ fanin_ptr, const int32_t *__restrict__ fanin_net,
                                      unsigned int *pending, int32_t *level, int32_t n_inputs, int32_t *next,
                                      unsigned int *next_size)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = frontier[i];
    for (int64_t k = fo_ptr[g]; k < fo_ptr[g + 1]; k++) {
        const int32_t t = fo[k];
        if (atomicSub(&pending[t], 1u) != 1u) continue;
        int32_t mx = 0;
        for (int64_t s = fanin_ptr[t]; s < fanin_ptr[t + 1]; s++) {
            const int32_t l = __hip_atomic_load(&level[fanin_net[s]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            mx = l > mx ? l : mx;
        }
        __hip_atomic_store(&level[n_inputs + t], mx + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        next[atomicAdd(next_size, 1u)] = t;
    }
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

hipError_t launch_fanout_count(const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t n_inputs, int32_t n_gates,
                               unsigned int *pending, unsigned int *fo_cnt, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(fanout_count_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, fanin_ptr, fanin_net,
                       n_inputs, n_gates, pending, fo_cnt);
    return hipGetLastError();
}

hipError_t launch_fanout_fill(const int64_t *fanin_ptr, const int32_t *fanin_net, int32_t n_inputs, int32_t n_gates,
                              const int64_t *fo_ptr, unsigned int *cursor, int32_t *fo, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(fanout_fill_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, fanin_ptr, fanin_net,
                       n_inputs, n_gates, fo_ptr, cursor, fo);
    return hipGetLastError();
}

hipError_t launch_level_seed(const unsigned int *pending, int32_t *level, int32_t n_inputs, int32_t n_gates,
                             int32_t *frontier, unsigned int *size, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(level_seed_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, pending, level, n_inputs,
                       n_gates, frontier, size);
    return hipGetLastError();
}

hipError_t launch_level_frontier(const int32_t *frontier, unsigned int n, const int64_t *fo_ptr, const int32_t *fo,
                                 const int64_t *fanin_ptr, const int32_t *fanin_net, unsigned int *pending,
                                 int32_t *level, int32_t n_inputs, int32_t *next, unsigned int *next_size,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(level_frontier_kernel, dim3((n + 255) / 256), dim3(256), 0, s, frontier, n, fo_ptr, fo,
                       fanin_ptr, fanin_net, pending, level, n_inputs, next, next_size);
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
// Arena reservation.  A wave reserves the words of its output chunks with
// one atomic on its stripe's counter.  When that stripe is full, up to 15
// other stripes spread over the arena (every stripe of a region with 16) are
// tried before the round is flagged for a retry (flags[0]), so one full
// stripe does not fail a round while others have room.  A failed try leaves its counter past the stripe's end (taking
// the words back could hand one range out twice while other waves reserve)
// and adds its words to the stripe's second counter, so that the host can
// tell the words handed out from the words lost to failed tries.  Returns
// the reservation's first word, counted from the window's `times`, or ~0
// when no try succeeded.
// --------------------------------------------------------------------------
constexpr uint32_t kStripeTries = 16;

// `pick` selects the first stripe (masked to the stripes there are); with
// dead nets released the reservation comes from region `region` of the
// window's table, whose entry is read here, at the reservation, so that its
// fields hold no registers through the rest of the wave's work.
__device__ __forceinline__ uint64_t arena_reserve(const WinView &win, uint32_t region, uint32_t pick, uint32_t n,
                                                  int lane)
{
    unsigned long long *bump = win.bump;
    uint64_t slice = win.slice_words, off = win.arena_off;
    uint32_t mask = win.stripe_mask;
    if (win.regions) {
        const ArenaRegion r = *kons(win.regions + region);
        bump = r.bump;
        slice = r.slice_words;
        off = r.off;
        mask = r.stripe_mask;
    }
    uint32_t s = pick & mask;
    // the first try inline; the rare further tries in a loop kept rolled,
    // so that the common path carries no extra registers
#pragma nounroll
    for (uint32_t k = 0; k < kStripeTries; k++) {
        uint64_t b = 0;
        if (lane == 0)
            b = __hip_atomic_fetch_add(glob(bump + (size_t)s * kBumpStride), (unsigned long long)n,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b = uniform64(b);
        if (b + n <= slice) return off + (uint64_t)s * slice + b;
        if (lane == 0)
            __hip_atomic_fetch_add(glob(bump + (size_t)s * kBumpStride + 1), (unsigned long long)n,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (mask == 0) break;
        s = (s + 97u) & mask;
    }
    if (lane == 0) __hip_atomic_fetch_or(glob(win.flags), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ~0ull;
}

// --------------------------------------------------------------------------
// Stimulus expansion (the input restructuring GATSPI does before its
// kernels, Section 4): absolute toggle times of input i become the
// (input, tile) chunks of the window, in cycle-local time, with every
// cycle's pre-cycle value in bit 15 of its lane end (and in the chunk
// mask).  Also adds the inputs' SAIF counts.
//
// One wave handles one input over an aligned group of kExpandGroup tiles.
// The group's toggles are one sorted range of the input's toggle list, and
// in the output they keep that order (cycle by cycle, which is lane after
// lane, chunk after chunk), so the wave writes them as one contiguous,
// coalesced range: lane k of a row handles toggle k.  Per-cycle counts come
// from an LDS histogram of the toggles' cycle indices.
// --------------------------------------------------------------------------

// Tiles an expansion wave handles: the chunks of one input in an aligned
// group of this many tiles are placed one after another in the arena, as
// gate evaluation places its output chunks, so that a consumer can copy a
// pin's group of chunks as one range.
constexpr uint32_t kExpandGroup = 4;

// First index in [a, b) whose value is >= key (b if none), searched by the
// whole wave: 64 samples per step narrow the range 64-fold.  Every lane
// gets the same result.
__device__ __forceinline__ int64_t wave_lower_bound(const int64_t *v, int64_t a, int64_t b, int64_t key, int lane)
{
    while (b - a > kLanes) {
        const int64_t stride = (b - a + kLanes - 1) / kLanes;
        const int64_t pos = a + (int64_t)lane * stride;
        const bool below = pos < b && *glob(v + pos) < key;
        const int c = __popcll(__ballot(below));           // the samples below key are a prefix
        if (c == 0) return a;
        const int64_t na = a + (int64_t)(c - 1) * stride + 1;
        const int64_t nb = a + (int64_t)c * stride;
        a = na;
        b = nb < b ? nb : b;
    }
    const bool below = a + lane < b && *glob(v + a + lane) < key;
    return a + __popcll(__ballot(below));
}

__global__ __launch_bounds__(256) void expand_kernel(StimView st, WinView win, SaifAcc acc, const int32_t *cycle0_p,
                                                     uint32_t salt, uint64_t n_waves)
{
    extern __shared__ uint32_t ex_hist[];                   // kExpandGroup * 64 counters per wave
    const int32_t cycle0 = *glob(cycle0_p);
    const int lane = threadIdx.x & (kLanes - 1);
    const uint32_t wib = uniform(threadIdx.x / kLanes);
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / kLanes) + wib;
    if (w >= n_waves) return;
    uint32_t *hist = ex_hist + wib * (kExpandGroup * kLanes);
    const uint32_t ntile = (uint32_t)win.n_tiles;
    const uint32_t ngrp = (ntile + kExpandGroup - 1) / kExpandGroup;
    const uint32_t i = uniform((uint32_t)(w / ngrp));
    const uint32_t t0 = uniform((uint32_t)(w % ngrp)) * kExpandGroup;
    const uint32_t nt = min(kExpandGroup, ntile - t0);
    const int64_t T = st.period;
    const int64_t lo = *kons(st.toggle_ptr + i), hi = *kons(st.toggle_ptr + i + 1);
    const uint32_t init_i = *kons(st.init + i) & 1u;
    // cycles [c_lo, c_hi) of the window, times [g0, g1)
    const int32_t c_lo = (int32_t)(t0 * kLanes);
    const int32_t c_hi = min((int32_t)((t0 + nt) * kLanes), win.n_cycles);
    const int64_t g0 = (int64_t)(cycle0 + c_lo) * T;
    const int64_t g1 = (int64_t)(cycle0 + c_hi) * T;
    const int64_t ga = wave_lower_bound(st.toggle_ps, lo, hi, g0, lane);
    const int64_t gz = wave_lower_bound(st.toggle_ps, ga, hi, g1, lane);
    const uint32_t n = (uint32_t)(gz - ga);

#pragma unroll
    for (uint32_t k = 0; k < kExpandGroup; k++) hist[k * kLanes + lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // one arena reservation for the group's chunks
    uint64_t base = 0;
    bool ok = true;
    if (n > 0) {
        base = arena_reserve(win, 0, blockIdx.x + salt, n, lane);     // region 0: the inputs
        ok = base != ~0ull;
    }
    // toggles, one per lane and row: cycle index (group-relative), local time,
    // the T1 term of the edge, and the group's output word
    const double inv_t = 1.0 / (double)T;
    int64_t s1 = 0;                                         // sum of -t (rising) / +t (falling) over edges
    for (uint32_t r = 0; r < n; r += kLanes) {
        const uint32_t k = r + (uint32_t)lane;
        if (k < n) {
            const int64_t t = *glob(st.toggle_ps + ga + k);
            const uint32_t d = (uint32_t)(t - g0);         // < kExpandGroup * 64 * T <= 2^32
            uint32_t cyc = (uint32_t)((double)d * inv_t);
            if ((uint64_t)cyc * (uint64_t)T > d) cyc--;     // the quotient from the reciprocal may be one high
            else if ((uint64_t)(cyc + 1) * (uint64_t)T <= d) cyc++;
            const int32_t tl = (int32_t)(d - cyc * (uint32_t)T);
            atomicAdd(&hist[cyc], 1u);
            if (ok) *glob(win.times + base + k) = tl;
            // value after this edge: the input's initial value flipped once per toggle so far
            const uint32_t after = init_i ^ (uint32_t)((ga + k - lo + 1) & 1);
            s1 += after ? -tl : tl;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    uint32_t before = 0;                                    // group toggles in earlier tiles
    uint32_t nact = 0;
    // the group's share of the input's glitch toggles; on a continuous view
    // it can be negative (below)
    int32_t glitch = 0;
    int64_t zt = 0;                                         // final values x T over the lane's cycles
    // Continuous segments of st.seg cycles (the window starts one): a
    // segment's glitch toggles are its toggles less the parity of their
    // number, i.e. less (toggles before its start XOR toggles before its
    // end) & 1.  The group counts its own toggles and subtracts that term
    // for the segments that end in it; pv is the parity term at the last
    // segment start seen (found by a search when the segment began before
    // the group).  A segment's toggles can all lie in an earlier group, so a
    // group's share can be negative; the shares of a segment's groups sum to
    // its count.
    const uint32_t S = st.seg > 1 ? (uint32_t)st.seg : 0u;
    uint32_t pv = 0, odd = 0;
    if (S) {
        const int32_t s0 = c_lo - (int32_t)((uint32_t)c_lo % S);
        const int64_t tb = s0 == c_lo ? ga : wave_lower_bound(st.toggle_ps, lo, ga, (int64_t)(cycle0 + s0) * T, lane);
        pv = (uint32_t)((tb - lo) & 1);
    }
    for (uint32_t u = 0; u < nt; u++) {
        const uint32_t tile = t0 + u;
        const bool active = (int32_t)(tile * kLanes) + lane < win.n_cycles;
        const uint32_t cnt = active ? hist[u * kLanes + lane] : 0u;
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = (uint32_t)lane63(incl);
        const uint32_t excl = before + incl - cnt;          // group toggles before this cycle
        const uint32_t init = active ? init_i ^ (uint32_t)((ga - lo + excl) & 1) : 0u;
        bool okc = ok;
        if (total > kMaxChunk) {
            if (lane == 0) __hip_atomic_fetch_or(glob(win.flags + 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            okc = false;
        }
        const uint64_t ci = (uint64_t)i * ntile + tile;
        *glob(win.ends + ci * kLanes + lane) = (uint16_t)((okc ? incl : 0u) | (init << kEndInitShift));
        const uint64_t mask = __ballot(init != 0);
        if (lane == 0) {
            ChunkHdr h;
            h.off = okc ? base + before : 0;
            h.mask = mask;
            *glob(win.hdr + ci) = h;
        }
        nact += (uint32_t)__popcll(__ballot(active));
        zt += active ? (int64_t)(init ^ (cnt & 1u)) * T : 0;
        if (S) {
            const uint32_t c = tile * kLanes + (uint32_t)lane;
            const uint64_t mb = __ballot(active && (int32_t)c > c_lo && c % S == 0u);
            const uint64_t mp = __ballot(((ga - lo + excl) & 1) != 0);
            for (uint64_t b = mb; b; b &= b - 1) {
                const uint32_t pb = (uint32_t)(mp >> __builtin_ctzll(b)) & 1u;
                odd += pv ^ pb;
                pv = pb;
            }
            glitch += (int32_t)total;
        } else {
            glitch += (int32_t)(total - (uint32_t)__popcll(__ballot(cnt & 1u)));   // all but one edge of odd lists
        }
        before += total;
    }
    if (S) {
        if ((uint32_t)c_hi % S == 0u) odd += pv ^ (uint32_t)((gz - lo) & 1);   // a segment ends with the group
        glitch -= (int32_t)odd;
    }
    const int64_t sum1 = wave_sum64(zt + s1);
    if (lane == 0) {
        __hip_atomic_fetch_add(glob(acc.tc + i), (unsigned long long)n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (glitch)                                         // sign-extended: a negative share subtracts
            __hip_atomic_fetch_add(glob(acc.ig + i), (unsigned long long)(int64_t)glitch, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(glob(acc.t1 + i), (unsigned long long)sum1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(glob(acc.t0 + i), (unsigned long long)((int64_t)nact * T - sum1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_expand(StimView st, WinView win, SaifAcc acc, const int32_t *cycle0, uint32_t salt, hipStream_t s)
{
    uint64_t n_waves = (uint64_t)st.n_inputs * (uint64_t)((win.n_tiles + kExpandGroup - 1) / kExpandGroup);
    if (n_waves == 0) return hipSuccess;
    const int wpb = 4;
    uint64_t blocks = (n_waves + wpb - 1) / wpb;
    const size_t lds = (size_t)wpb * kExpandGroup * kLanes * sizeof(uint32_t);
    hipLaunchKernelGGL(expand_kernel, dim3((unsigned)blocks), dim3(64 * wpb), lds, s, st, win, acc, cycle0, salt,
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
extern __shared__ int32_t gs_lds[];

// chunk[idx] with a 32-bit byte offset from a wave-uniform base, so the
// load can use the scalar-base + vector-offset addressing mode
__device__ __forceinline__ int32_t ld_word(const int32_t *chunk, uint32_t idx)
{
    return *(const GAS int32_t *)((const GAS char *)glob(chunk) + (uint64_t)(idx << 2));
}

// base[idx] = v for a wave-uniform base (scalar base + 32-bit vector offset)
__device__ __forceinline__ void st_word(int32_t *base, uint32_t idx, int32_t v)
{
    *(GAS int32_t *)((GAS char *)glob(base) + (uint64_t)(idx << 2)) = v;
}

__device__ __forceinline__ void st_u16(uint16_t *base, uint32_t idx, uint16_t v)
{
    *(GAS uint16_t *)((GAS char *)glob(base) + (uint64_t)(idx << 1)) = v;
}

// base[idx] for a wave-uniform base (scalar base + 32-bit vector offset)
__device__ __forceinline__ uint32_t ld_u16(const uint16_t *base, uint32_t idx)
{
    return *(const GAS uint16_t *)((const GAS char *)glob(base) + (uint64_t)(idx << 1));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)l);
    return ((uint64_t)hi << 32) | lo;
}

// Arc data of one gate's pins (wave-uniform).
template <int K>
struct Arcs {
    int32_t q[K], d[K][8], wr[K], wf[K];

    // Pin j's arc delay for output value y in pin state st (after the
    // switch).  Arithmetic selects: a select between array elements would
    // become an address select and force the arrays to scratch.
    __device__ __forceinline__ int32_t pin_delay(int j, uint32_t st, int y) const
    {
        const int32_t mc = -(int32_t)((st >> q[j]) & 1), me = -(int32_t)((st >> j) & 1), mo = -(int32_t)y;
        int32_t v[4];
#pragma unroll
        for (int i = 0; i < 4; i++) v[i] = d[j][i] + (mc & (d[j][i + 4] - d[j][i]));   // condition value
        const int32_t f = v[0] + (me & (v[2] - v[0]));                                   // input edge
        const int32_t r = v[1] + (me & (v[3] - v[1]));
        return f + (mo & (r - f));                                                       // output edge
    }

    // Smallest arc delay over the pins in sw for output value y, in pin
    // state st (gates with more than three pins; smaller gates read it from
    // the wave's lookup table).
    __device__ __forceinline__ int32_t delay(uint32_t st, uint32_t sw, int y) const
    {
        int32_t dm = kInf;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const int32_t dj = pin_delay(j, st, y);
            const int32_t m = -(int32_t)((sw >> j) & 1);
            dm = min(dm, (dj & m) | (kInf & ~m));
        }
        return dm;
    }
};

// Per-lane cursor over one gate's fanin lists in one cycle: pin j's next
// event is word idx[j] of its chunk (a[j] = its arrival time).  LDSRC: the
// chunk was staged in LDS by the wave and starts at word base[j] of the
// wave's LDS; otherwise it is read from the transition arena at chunk[j].
template <int K, bool WIRES, bool LDSRC>
struct Cursor {
    const int32_t *chunk[K];
    uint32_t base[K];
    uint32_t idx[K], end[K];
    int32_t a[K];
    uint32_t state;
    bool transport;                 // wire delays without the net-delay filter

    __device__ __forceinline__ int32_t word(int j, uint32_t i) const
    {
        if (LDSRC) return gs_lds[base[j] + i];
        return ld_word(chunk[j], i);
    }

    __device__ __forceinline__ void advance(const Arcs<K> &arc, int j)
    {
        if (!WIRES && LDSRC) {
            // an LDS read past the lane's words stays inside the LDS
            // allocation or returns 0, so it needs no branch
            const int32_t v = word(j, idx[j]);
            a[j] = idx[j] < end[j] ? v : kInf;
            return;
        }
        if (!WIRES) {
            a[j] = idx[j] < end[j] ? word(j, idx[j]) : kInf;
            return;
        }
        const int pv = (state >> j) & 1;
        const int32_t d = pv ? arc.wf[j] : arc.wr[j];       // the net edge goes to !pv
        const int32_t d1 = pv ? arc.wr[j] : arc.wf[j];      // the edge after it goes back to pv
        // the pair is dropped when the second edge comes before the first
        // arrives (inertial filter), or without the filter when the second
        // arrives no later than the first (transport delay)
        const int32_t thr = transport ? d - d1 + 1 : d;
        for (;;) {
            if (idx[j] >= end[j]) {
                a[j] = kInf;
                return;
            }
            const int32_t e0 = word(j, idx[j]);
            if (idx[j] + 1 < end[j] && word(j, idx[j] + 1) - e0 < thr) {
                idx[j] += 2;                                // the pulse vanishes
                continue;
            }
            a[j] = e0 + d;
            return;
        }
    }
};

// Lookup table of a gate with up to three pins, one entry per (pin state
// after an event, mask of the pins that switched): bit 0 = the truth-table
// output, bits 1.. = the smallest arc delay of the switched pins for that
// output edge.  64 words per wave in LDS, built by the 64 lanes at once.
template <int K>
__device__ __forceinline__ void build_lut(const Arcs<K> &arc, uint64_t truth, int lane, uint32_t lut_base)
{
    const uint32_t st = (uint32_t)lane >> 3, m = (uint32_t)lane & 7u;
    const int y = (int)((truth >> st) & 1);
    int32_t d = kInf >> 1;
#pragma unroll
    for (int j = 0; j < K; j++) {
        const int32_t dj = arc.pin_delay(j, st, y);
        const int32_t mj = -(int32_t)((m >> j) & 1);
        d = min(d, (dj & mj) | ((kInf >> 1) & ~mj));
    }
    gs_lds[lut_base + lane] = (d << 1) | y;
}

// One walk over a lane's fanin lists (Algorithm 1's event loop).  MODE 0
// stages output edges in LDS (at most CAP per lane); MODE 1 writes them to
// dst[0 .. keep) in global memory (entries at or beyond `keep` are retracted
// before the walk ends, or are the edge a continuous segment carries into
// the next cycle, so they are not stored).  w0 >= 0: the output has an edge
// to z pending at w0 when the lane starts (carried from the cycle before;
// the output is !z until then).  w_out: the time of the list's last edge.
template <int K, bool WIRES, bool LDSRC, int MODE, int CAP>
__device__ __forceinline__ void walk(Cursor<K, WIRES, LDSRC> &P, const Arcs<K> &arc, uint64_t truth, int32_t T,
                                     int z, uint32_t lut_base, uint32_t out_lane, int32_t *dst, int32_t keep,
                                     int32_t w0, int32_t &cnt_out, int32_t &acc_out, int32_t &z_out, int32_t &w_out)
{
#pragma unroll
    for (int j = 0; j < K; j++) P.advance(arc, j);
    int32_t W = 0, Wp = 0, cnt = 0, acc = 0;
    if (w0 >= 0) {
        if (MODE == 0) {
            if (CAP > 0) gs_lds[out_lane] = w0;
        } else {
            if (keep > 0) *glob(dst) = w0;
        }
        const int32_t ce = min(w0, T);
        acc += z ? -ce : ce;
        cnt = 1;
        W = w0;
    }
    for (;;) {
        int32_t t = P.a[0];
#pragma unroll
        for (int j = 1; j < K; j++) t = min(t, P.a[j]);
        if (t == kInf) break;
        uint32_t sw = 0;
#pragma unroll
        for (int j = 0; j < K; j++) {
            if (P.a[j] == t) {
                sw |= 1u << j;
                P.state ^= 1u << j;             // the wire filter reads the pin's new value
                P.idx[j]++;
                P.advance(arc, j);
            }
        }
        int y;
        int32_t d;
        if (K <= 3) {
            const int32_t ent = gs_lds[lut_base + ((P.state << 3) | sw)];
            y = ent & 1;
            d = ent >> 1;
        } else {
            y = (int)((truth >> P.state) & 1);
            d = 0;
        }
        if (y != z) {
            if (K > 3) d = arc.delay(P.state, sw, y);
            const bool retract = t < W;
            const int32_t e = retract ? W : t + d;
            const int32_t ce = min(e, T);
            acc += y ? -ce : ce;
            if (retract) {
                cnt--;
                W = Wp;
            } else {
                if (MODE == 0) {
                    if (cnt < CAP) gs_lds[out_lane + cnt * kLanes] = t + d;
                } else {
                    if (cnt < keep) *glob(dst + cnt) = t + d;
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
    w_out = W;
}

// Interconnect filter (Algorithm 1, net-delay filtering) applied to one
// lane's staged list of a pin, in place: walking the net's edges in order, an
// edge followed by the next one sooner than the wire delay of the value it
// goes to is dropped together with that next edge; every other edge becomes
// a pin arrival at its time plus that delay.  With transport delays (the
// filter deleted) a pair is dropped only when the next edge's arrival is no
// later than this one's.  v is the net's value before the first edge.  On
// return [lo, hi) holds the arrivals.  Written without branches: a lane
// writes behind its own read position only, and the word read past its list
// (another lane's, or outside the stage) is never used.
__device__ __forceinline__ void wire_filter_lds(uint32_t base, uint32_t lo, uint32_t &hi, uint32_t v, int32_t wr,
                                                int32_t wf, bool transport)
{
    uint32_t r = lo, o = lo;
    while (r < hi) {
        const int32_t e0 = gs_lds[base + r];
        const int32_t e1 = gs_lds[base + r + 1];
        const uint32_t nv = v ^ 1u;
        const int32_t d = nv ? wr : wf;
        const int32_t d1 = nv ? wf : wr;
        const int32_t thr = transport ? d - d1 + 1 : d;
        const bool drop = r + 1 < hi && e1 - e0 < thr;
        gs_lds[base + o] = e0 + d;
        o += drop ? 0u : 1u;
        r += drop ? 2u : 1u;
        v = drop ? v : nv;
    }
    hi = o;
}

// The event loop of `walk` for fanin words staged in LDS without
// interconnect delays, written without branches: every pin's next word and
// every state update is computed for all lanes and selected, so that a
// lane's event costs the same straight-line code whichever pins switch and
// whether the output edge is appended, cancelled or not needed.  Output
// edges go to LDS slot min(cnt, CAP); slot CAP is a spare that absorbs the
// stores of steps that append nothing and of lanes past CAP.  w0 and w_out
// as in `walk`.
template <int K, int CAP>
__device__ __forceinline__ void walk_lds(Cursor<K, false, true> &P, const Arcs<K> &arc, uint64_t truth, int32_t T,
                                         int z, uint32_t lut_base, uint32_t out_lane, int32_t w0, int32_t &cnt_out,
                                         int32_t &w_out)
{
#pragma unroll
    for (int j = 0; j < K; j++) {
        const int32_t v = gs_lds[P.base[j] + P.idx[j]];
        P.a[j] = P.idx[j] < P.end[j] ? v : kInf;
    }
    int32_t W = 0, Wp = 0, cnt = 0;
    if (w0 >= 0) {
        gs_lds[out_lane] = w0;
        cnt = 1;
        W = w0;
    }
    for (;;) {
        int32_t t = P.a[0];
#pragma unroll
        for (int j = 1; j < K; j++) t = min(t, P.a[j]);
        if (t == kInf) break;
        uint32_t sw = 0;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const uint32_t m = P.a[j] == t ? 1u : 0u;
            sw |= m << j;
            P.idx[j] += m;
        }
        P.state ^= sw;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const int32_t v = gs_lds[P.base[j] + P.idx[j]];
            P.a[j] = P.idx[j] < P.end[j] ? v : kInf;
        }
        int y;
        int32_t d;
        if (K <= 3) {
            const int32_t ent = gs_lds[lut_base + ((P.state << 3) | sw)];
            y = ent & 1;
            d = ent >> 1;
        } else {
            y = (int)((truth >> P.state) & 1);
            d = arc.delay(P.state, sw, y);
        }
        const bool chg = y != z;
        const bool retract = t < W;
        const int32_t td = t + d;
        gs_lds[out_lane + min(cnt, CAP) * kLanes] = td;
        const bool app = chg && !retract;
        cnt += app ? 1 : (chg ? -1 : 0);
        const int32_t W0 = W;
        W = app ? td : (chg ? Wp : W);
        Wp = app ? W0 : Wp;
        z = y;
    }
    cnt_out = cnt;
    w_out = W;
}

// The event loop of walk_lds for a queued lane of the compacted path: the
// lane's pin lists are staged at absolute LDS positions [idx, end), and its
// output edges go to LDS slots opos, opos + 1, ...  A lane appends at most
// one edge per event time, so the slot written in a step (the current count,
// also when nothing is appended) stays below the lane's event count, inside
// the region reserved for it.
template <int K>
__device__ __forceinline__ void walk_lds_c(Cursor<K, false, true> &P, int z, uint32_t lut_base, uint32_t opos,
                                           int32_t &cnt_out)
{
#pragma unroll
    for (int j = 0; j < K; j++) {
        const int32_t v = gs_lds[P.idx[j]];
        P.a[j] = P.idx[j] < P.end[j] ? v : kInf;
    }
    int32_t W = 0, Wp = 0, cnt = 0;
    for (;;) {
        int32_t t = P.a[0];
#pragma unroll
        for (int j = 1; j < K; j++) t = min(t, P.a[j]);
        if (t == kInf) break;
        uint32_t sw = 0;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const uint32_t m = P.a[j] == t ? 1u : 0u;
            sw |= m << j;
            P.idx[j] += m;
        }
        P.state ^= sw;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const int32_t v = gs_lds[P.idx[j]];
            P.a[j] = P.idx[j] < P.end[j] ? v : kInf;
        }
        const int32_t ent = gs_lds[lut_base + ((P.state << 3) | sw)];
        const int y = ent & 1;
        const int32_t td = t + (ent >> 1);
        const bool chg = y != z;
        const bool retract = t < W;
        gs_lds[opos + (uint32_t)cnt] = td;
        const bool app = chg && !retract;
        cnt += app ? 1 : (chg ? -1 : 0);
        const int32_t W0 = W;
        W = app ? td : (chg ? Wp : W);
        Wp = app ? W0 : Wp;
        z = y;
    }
    cnt_out = cnt;
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Compacted evaluation of one staged tile group of a gate with up to three
// pins (lane = cycle of a tile, GT tiles).  Most (gate, cycle) lanes see no
// pin event or exactly one, and the per-tile walk runs as long as the
// busiest lane of the tile; here the work is split by event count:
//   1. per tile: a lane without pin events keeps its settled value and has
//      no output edge; a lane with exactly one takes Algorithm 1's step in
//      closed form (the pin switches at its arrival time, the truth table
//      gives the new value, and an output edge is appended at that time plus
//      the arc delay iff the value changes); a lane with two or more is
//      queued with its pin ranges in the stage;
//   2. the queued lanes of all GT tiles are walked together, 64 per pass,
//      with interconnect filtering first when the design has wires; each
//      writes its edges to its own region of the output stage;
//   3. per tile: the lane counts are prefix-summed; the group reserves the
//      exact number of output words with one atomic; lane ends, chunk
//      headers and single edges are written, and the queued lanes copy their
//      edges out in one more pass.
// The SAIF terms of every lane are added to the caller's sums.  Returns
// false, having written nothing outside the wave's LDS, when more than
// kQueueCap lanes of the group have two or more events.
template <int K, bool WIRES, uint32_t GT>
__device__ __forceinline__ bool compact_group(const WinView &win, const Arcs<K> &arc, uint64_t truth, uint32_t out_row,
                                              uint32_t tile_g, uint32_t ng, int lane, uint32_t lut_base,
                                              uint32_t out_base, uint32_t c_pos, const uint32_t (&ev)[K][GT / 2],
                                              uint32_t salt, bool transport, uint32_t &tc_sum, uint32_t &ig_sum,
                                              uint32_t &nact_sum, int32_t &t1_lane, uint32_t region)
{
    const int32_t T = win.period;
    const uint32_t ntile = (uint32_t)win.n_tiles;
    const uint32_t queue = out_base + kOutStageWords;
    const uint32_t stage_base = out_base - kStageWords;
    uint64_t mmask[GT];           // lanes queued in tile u
    uint32_t qbase[GT];           // their first queue entry
    int32_t e1[GT];               // a single-event lane's output edge
    uint32_t bits = 0;            // bit u: that edge exists; bit GT + u: settled output value at t = 0
    uint32_t qn = 0, tileoff = 0;

    // 1. classify the lanes of every tile
#pragma unroll
    for (uint32_t u = 0; u < GT; u++) {
        mmask[u] = 0;
        qbase[u] = qn;
        e1[u] = 0;
        if (u < ng) {
            uint32_t hi[K], lo[K], nj[K], pos[K];
            uint32_t st0 = 0, nev = 0, lsum = 0;
#pragma unroll
            for (int j = 0; j < K; j++) {
                const uint32_t w = (ev[j][u / 2] >> (16 * (u & 1))) & 0xffffu;
                hi[j] = w & kEndCount;
                lo[j] = wave_shr1(hi[j]);
                nj[j] = hi[j] - lo[j];
                st0 |= (w >> kEndInitShift) << j;
                nev += nj[j];
                lsum += lo[j];
                pos[j] = (uint32_t)__builtin_amdgcn_readlane((int)c_pos, j * (int)GT + (int)u) + lo[j];
            }
            const uint32_t y0 = (uint32_t)(truth >> st0) & 1u;
            // one event: the first pin with an event is the one
            // (the wire delay by the pin's new value, selected arithmetically:
            // a select between array elements would become an address select
            // and force the arc arrays to scratch)
            uint32_t p1 = pos[K - 1], sw = 1u << (K - 1);
            int32_t dw = 0;
            if (WIRES) {
                const int32_t m = -(int32_t)((st0 >> (K - 1)) & 1u);
                dw = arc.wr[K - 1] + (m & (arc.wf[K - 1] - arc.wr[K - 1]));
            }
#pragma unroll
            for (int j = K - 2; j >= 0; j--) {
                const bool h = nj[j] != 0;
                p1 = h ? pos[j] : p1;
                sw = h ? 1u << j : sw;
                if (WIRES) {
                    const int32_t m = -(int32_t)((st0 >> j) & 1u);
                    const int32_t dj = arc.wr[j] + (m & (arc.wf[j] - arc.wr[j]));
                    dw = h ? dj : dw;
                }
            }
            const int32_t ta = gs_lds[p1] + dw;
            const int32_t ent = gs_lds[lut_base + (((st0 ^ sw) << 3) | sw)];
            const bool edge = nev == 1 && (uint32_t)(ent & 1) != y0;
            e1[u] = ta + (ent >> 1);
            bits |= (edge ? 1u << u : 0u) | (y0 << (GT + u));
            // two or more: queue the lane
            const bool multi = nev >= 2;
            const uint64_t mm = __ballot(multi);
            const uint32_t nm = (uint32_t)__popcll(mm);
            if (qn + nm > kQueueCap) return false;
            if (multi) {
                const uint32_t q = qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
                const uint32_t qa = queue + q * (uint32_t)K;
                // K words: pin j's list as stage-relative [start, end) in
                // bits 0-9 and 10-19; word 0 also carries the lane's output
                // region (from out_base) and its pin state in bits 20-31
#pragma unroll
                for (int j = 0; j < K; j++) {
                    const uint32_t r = pos[j] - stage_base;
                    uint32_t w = r | ((r + nj[j]) << 10);
                    if (j == 0) w |= ((tileoff + lsum) | (st0 << 9)) << 20;
                    gs_lds[qa + j] = (int32_t)w;
                }
            }
            mmask[u] = mm;
            qn += nm;
#pragma unroll
            for (int j = 0; j < K; j++) tileoff += (uint32_t)lane63(hi[j]);
        }
    }
    wave_lds_sync();

    // 2. walk the queued lanes, 64 at a time
    for (uint32_t qb = 0; qb < qn; qb += kLanes) {
        const uint32_t q = qb + (uint32_t)lane;
        const bool valid = q < qn;
        const uint32_t qa = queue + min(q, qn - 1) * (uint32_t)K;
        Cursor<K, false, true> P;
        uint32_t info = 0;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const uint32_t w = (uint32_t)gs_lds[qa + j];
            if (j == 0) info = w >> 20;
            P.base[j] = 0;
            P.idx[j] = stage_base + (w & 0x3ffu);
            P.end[j] = valid ? stage_base + ((w >> 10) & 0x3ffu) : P.idx[j];
        }
        P.state = (info >> 9) & 7u;
        P.transport = transport;
        if (WIRES) {
#pragma unroll
            for (int j = 0; j < K; j++)
                wire_filter_lds(0, P.idx[j], P.end[j], (P.state >> j) & 1u, arc.wr[j], arc.wf[j], transport);
        }
        int32_t cnt;
        walk_lds_c<K>(P, (int)((truth >> ((info >> 9) & 7u)) & 1u), lut_base, out_base + (info & 0x1ffu), cnt);
        if (valid) gs_lds[qa] = (int32_t)((info << 20) | (uint32_t)cnt);       // count in bits 0-9
    }
    wave_lds_sync();

    // 3a. lane counts, their prefix sums and the group's exact total
    uint32_t incl[GT];
    uint32_t tot[GT];
    uint32_t R = 0;
#pragma unroll
    for (uint32_t u = 0; u < GT; u++) {
        incl[u] = 0;
        tot[u] = 0;
        if (u < ng) {
            const uint64_t mm = mmask[u];
            const bool multi = (mm >> lane) & 1u;
            uint32_t c = (bits >> u) & 1u;
            if (multi) {
                const uint32_t q = qbase[u] + __builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
                c = (uint32_t)gs_lds[queue + q * (uint32_t)K] & 0x3ffu;
            }
            incl[u] = wave_incl_scan(c);
            tot[u] = (uint32_t)lane63(incl[u]);
            ig_sum += tot[u] - (uint32_t)__popcll(__ballot(c & 1u));
            R += tot[u];
        }
    }
    tc_sum += R;

    // one reservation for the group's output chunks, exactly their words
    uint64_t wbase = 0;
    bool ok = true;
    if (R > 0) {
        wbase = arena_reserve(win, region, blockIdx.x + salt, R, lane);
        ok = wbase != ~0ull;
        if (!ok) wbase = 0;
    }
    int32_t *out = win.times + wbase;

    // 3b. lane ends, headers, single edges; queued lanes learn their place
    uint32_t rel = 0;
#pragma unroll
    for (uint32_t u = 0; u < GT; u++) {
        if (u < ng) {
            const uint32_t tile = tile_g + u;
            const int32_t first_cycle = (int32_t)(tile * kLanes);
            const bool active = first_cycle + lane < win.n_cycles;
            const uint32_t y0 = (bits >> (GT + u)) & 1u;
            const uint32_t one = (bits >> u) & 1u;
            const uint64_t ci = (uint64_t)out_row * ntile + tile;
            const uint32_t yb = active ? y0 : 0u;
            st_u16(win.ends + ci * kLanes, (uint32_t)lane, (uint16_t)((ok ? incl[u] : 0u) | (yb << kEndInitShift)));
            const uint64_t mask = __ballot(yb != 0);
            if (lane == 0) {
                ChunkHdr h;
                h.off = ok ? wbase + rel : 0;
                h.mask = mask;
                *glob(win.hdr + ci) = h;
            }
            const uint32_t first = rel + wave_shr1(incl[u]);
            if (ok && one) st_word(out, first, e1[u]);
            const uint64_t mm = mmask[u];
            const bool multi = (mm >> lane) & 1u;
            if (multi) {
                const uint32_t q = qbase[u] + __builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
                const uint32_t a = queue + q * (uint32_t)K;
                gs_lds[a] = (int32_t)(((uint32_t)gs_lds[a] & 0xfff003ffu) | (first << 10));   // first word in bits 10-19
            } else if (active) {
                // T1 of the cycle: the settled value over [0, T), or up to
                // the single edge and the new value after it
                const int32_t ce = min(e1[u], T);
                t1_lane += one ? (y0 ? ce : T - ce) : (int32_t)y0 * T;
            }
            const int32_t na = win.n_cycles - first_cycle;
            nact_sum += (uint32_t)(na < 0 ? 0 : (na > kLanes ? kLanes : na));
            rel += tot[u];
        }
    }
    wave_lds_sync();

    // 3c. queued lanes copy their edges out and add their T1 terms
    for (uint32_t qb = 0; qb < qn; qb += kLanes) {
        const uint32_t q = qb + (uint32_t)lane;
        const bool valid = q < qn;
        const uint32_t w0 = (uint32_t)gs_lds[queue + min(q, qn - 1) * (uint32_t)K];
        const int32_t c = valid ? (int32_t)(w0 & 0x3ffu) : 0;
        const uint32_t first = (w0 >> 10) & 0x3ffu;
        const uint32_t opos = out_base + ((w0 >> 20) & 0x1ffu);
        int v = (int)((truth >> ((w0 >> 29) & 7u)) & 1u);
        int32_t s1 = 0;
        for (int32_t i = 0; i < c; i++) {
            const int32_t e = gs_lds[opos + (uint32_t)i];
            if (ok) st_word(out, first + (uint32_t)i, e);
            v ^= 1;
            const int32_t ce = min(e, T);
            s1 += v ? -ce : ce;
        }
        if (valid) t1_lane += v * T + s1;
    }
    return true;
}

// One gate over `ntl` consecutive tiles starting at tile0 (one lane per
// cycle of a tile).  The per-gate work (arc data, delay table) is done once.
// Tiles are processed in groups of GT: lane c = j * GT + u fetches the
// header and the edge total of pin j's chunk in tile u of the group, every
// lane fetches its own lane ends of all the group's chunks, and the group's
// fanin words are then copied into LDS, so that the walks read no global
// memory (groups too large for the staging area walk the arena instead).
// SAIF counts of the output net are summed over the tiles and added with
// one atomic per counter.
template <int K, bool WIRES, int CAP, bool REMAP, bool CONT>
__device__ __forceinline__ void eval_gate(const Seg &sg, const GateRec &g, uint32_t tile0, uint32_t ntl, int lane,
                                          uint32_t lut_base, uint32_t out_base, uint32_t stage_base)
{
    static_assert(!(CONT && (WIRES || REMAP)), "continuous segments: designs without interconnect delays, whole windows");
    constexpr uint32_t GT = K <= 3 ? 4 : 2;
    const WinView &win = sg.win;
    const bool transport = (sg.mode & 1u) != 0;
    const int32_t T = win.period;
    const uint32_t ntile = (uint32_t)win.n_tiles;
    Arcs<K> arc;
    // chunk row of every fanin and of the output: the net id, or its slot
    // in the re-simulated cone (REMAP; then rd_* marks a resident chunk)
    uint32_t row[K];
    bool resident[K];
    uint32_t out_row = g.out;
    if (REMAP) out_row = (uint32_t)*kons(win.slot + g.out);
#pragma unroll
    for (int j = 0; j < K; j++) {
        const PinRec pr = *kons(sg.pins + g.pin0 + j);
        row[j] = (uint32_t)pr.net;
        resident[j] = false;
        if (REMAP) {
            const int32_t sl = *kons(win.slot + pr.net);
            resident[j] = sl < 0;
            row[j] = sl < 0 ? (uint32_t)pr.net : (uint32_t)sl;
        }
        arc.q[j] = pr.q;
#pragma unroll
        for (int i = 0; i < 8; i++) arc.d[j][i] = pr.d[i];
        arc.wr[j] = pr.wr; arc.wf[j] = pr.wf;
    }
    if (K <= 3) {
        build_lut<K>(arc, g.truth, lane, lut_base);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the chunk this lane fetches the header of
    const uint32_t cj = (uint32_t)lane / GT, cu = (uint32_t)lane % GT;
    uint32_t crow = 0;
    bool cres = false;
#pragma unroll
    for (int j = 0; j < K; j++) {
        if (cj == (uint32_t)j) {
            crow = row[j];
            cres = resident[j];
        }
    }
    const ChunkHdr *chsrc = (REMAP && cres) ? win.rd_hdr : win.hdr;
    const uint16_t *cesrc = (REMAP && cres) ? win.rd_ends : win.ends;

    const uint32_t out_lane = out_base + lane;
    uint32_t tc_sum = 0, nact_sum = 0, ig_sum = 0;
    int32_t t1_lane = 0;
    // continuous segments of seg_len cycles (the wave's first tile starts
    // one): the edge carried into the next lane, and the output's value at
    // the start of the open segment
    const uint32_t seg_len = CONT ? (sg.mode >> 8) : 1u;
    int32_t carry = -1;
    uint32_t seg_y = 0;
    for (uint32_t gb = 0; gb < ntl; gb += GT) {
        const uint32_t ng = min(GT, ntl - gb);
        // Every load below is issued by every lane (lanes without a chunk of
        // their own, and tiles past a ragged group's end, read the group's
        // last chunk again), so that the wait for the first of them does not
        // have to cover the others.
        const bool cval = cj < (uint32_t)K && cu < ng;
        const uint64_t cci = (uint64_t)crow * ntile + tile0 + gb + min(cu, ng - 1);
        const ChunkHdr ch = *glob(chsrc + cci);
        const uint32_t c_tot = cval ? (uint32_t)*glob(cesrc + cci * kLanes + kLanes - 1) & kEndCount : 0u;
        const uint64_t c_off = ch.off;
        // lane ends of pin j in tiles u and u+1 of the group share one word
        uint32_t ev[K][GT / 2];
#pragma unroll
        for (int j = 0; j < K; j++) {
            const uint16_t *esrc = (REMAP && resident[j]) ? win.rd_ends : win.ends;
#pragma unroll
            for (uint32_t u = 0; u < GT; u += 2) {
                const uint16_t *r0 = esrc + ((uint64_t)row[j] * ntile + tile0 + gb + min(u, ng - 1)) * kLanes;
                const uint16_t *r1 = esrc + ((uint64_t)row[j] * ntile + tile0 + gb + min(u + 1, ng - 1)) * kLanes;
                ev[j][u / 2] = ld_u16(r0, (uint32_t)lane) | (ld_u16(r1, (uint32_t)lane) << 16);
            }
        }
        // The group's fanin words (the stage size it needs): a lane's output
        // never has more edges than its pins have events (Algorithm 1
        // appends at most one edge per event), so they also bound its output.
        const uint32_t c_incl = wave_incl_scan(c_tot);
        const uint32_t bound = (uint32_t)lane63(c_incl);
        const uint32_t c_pos = stage_base + wave_shr1(c_incl);  // chunk's first word in the LDS stage
        const uint32_t pick = blockIdx.x + sg.salt;           // the arena stripe (see arena_reserve)
        const bool staged = bound <= kStageWords;
        // staged groups of gates with up to three pins take the compacted
        // path, which reserves exactly its output words later
        const bool try_compact = K <= 3 && staged && !CONT;
        if (!staged && lane == 0)                               // counted for the statistics
            __hip_atomic_fetch_add(glob(win.flags + 4), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // A producing wave places the chunks of its tile group one after
        // another, so a pin's chunks in this group are usually one
        // contiguous range of the arena, and the stage keeps them in the same
        // order: then each pin is copied as one range.
        const uint32_t nlo = dpp0<0x101>((uint32_t)c_off), nhi = dpp0<0x101>((uint32_t)(c_off >> 32));   // row_shl:1
        const bool gap = cval && cu + 1 < ng && c_off + c_tot != (((uint64_t)nhi << 32) | nlo);
        const bool runs = __ballot(gap) == 0;
        if (staged && bound > 0 && runs) {
            uint32_t pin_pos[K], pin_n[K];
#pragma unroll
            for (int j = 0; j < K; j++) {
                pin_pos[j] = (uint32_t)__builtin_amdgcn_readlane((int)c_pos, j * (int)GT);
                const uint32_t pend = j + 1 < K ? (uint32_t)__builtin_amdgcn_readlane((int)c_pos, (j + 1) * (int)GT)
                                                : stage_base + bound;
                pin_n[j] = pend - pin_pos[j];
            }
            int32_t v0[K], v1[K];
#pragma unroll
            for (int j = 0; j < K; j++) {
                const int32_t *src = win.times + readlane64(c_off, (uint32_t)j * GT);
                v0[j] = (uint32_t)lane < pin_n[j] ? ld_word(src, (uint32_t)lane) : 0;
                v1[j] = (uint32_t)lane + kLanes < pin_n[j] ? ld_word(src, (uint32_t)lane + kLanes) : 0;
            }
#pragma unroll
            for (int j = 0; j < K; j++) {
                if ((uint32_t)lane < pin_n[j]) gs_lds[pin_pos[j] + lane] = v0[j];
                if ((uint32_t)lane + kLanes < pin_n[j]) gs_lds[pin_pos[j] + kLanes + lane] = v1[j];
            }
#pragma unroll
            for (int j = 0; j < K; j++) {
                if (pin_n[j] > 2 * kLanes) {
                    const int32_t *src = win.times + readlane64(c_off, (uint32_t)j * GT);
                    for (uint32_t r = 2 * kLanes + lane; r < pin_n[j]; r += kLanes)
                        gs_lds[pin_pos[j] + r] = ld_word(src, r);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else if (staged && bound > 0) {
            // chunks scattered over the arena: copied one by one
            for (uint32_t c = 0; c < K * GT; c++) {
                const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)c_tot, (int)c);
                const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)c_pos, (int)c);
                const int32_t *src = win.times + readlane64(c_off, c);
                for (uint32_t r = lane; r < n; r += kLanes) gs_lds[p + r] = ld_word(src, r);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if constexpr (K <= 3) {
            if (try_compact) {
                if (compact_group<K, WIRES, GT>(win, arc, g.truth, out_row, tile0 + gb, ng, lane, lut_base, out_base,
                                                c_pos, ev, sg.salt, transport, tc_sum, ig_sum, nact_sum, t1_lane,
                                                g.dead))
                    continue;
                // too many lanes with two or more events: the per-tile walk
                if (lane == 0)
                    __hip_atomic_fetch_add(glob(win.flags + 5), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // the per-tile walk.  A staged group (at most kStageWords fanin
        // words, which bound its output) reserves that bound at once, so the
        // atomic's latency overlaps the walk; an unstaged group, where
        // activity is dense and memory matters, reserves each tile's exact
        // words once the tile's lane counts are known.
        // On a continuous view an edge carried into the group's first lane
        // can add one edge (carries only move edges between the group's
        // lanes, or out of it).
        const uint32_t obound = bound + (CONT ? 1u : 0u);
        uint64_t gbase = 0;                                     // staged: the group's reservation
        bool gok = true;
        uint32_t used = 0;                                      // staged: its words handed out
        if (staged && obound > 0) {
            gbase = arena_reserve(win, g.dead, pick, obound, lane);
            gok = gbase != ~0ull;
        }
        for (uint32_t u = 0; u < ng; u++) {
            const uint32_t tile = tile0 + gb + u;
            const int32_t lc = (int32_t)(tile * kLanes) + lane;
            const bool active = lc < win.n_cycles;
            // A lane past the window's last cycle has an empty list in every
            // chunk (its lane end repeats the one before), so it walks nothing.
            uint32_t lo[K], hi[K], base[K];
            uint32_t state0 = 0;
#pragma unroll
            for (int j = 0; j < K; j++) {
                const uint32_t c = (uint32_t)j * GT + u;
                base[j] = (uint32_t)__builtin_amdgcn_readlane((int)c_pos, (int)c);
                hi[j] = ev[j][0] & kEndCount;
                lo[j] = wave_shr1(hi[j]);
                state0 |= ((ev[j][0] >> kEndInitShift) & 1u) << j;
            }
            // A group too large for the stage whose tile alone fits it: the
            // tile's fanin chunks are copied in, so that its walk reads LDS
            // too (its output words are still reserved per tile).
            bool lstaged = staged;
            if (!staged) {
                uint32_t tn[K], tsum = 0;
#pragma unroll
                for (int j = 0; j < K; j++) {
                    tn[j] = (uint32_t)__builtin_amdgcn_readlane((int)c_tot, j * (int)GT + (int)u);
                    tsum += tn[j];
                }
                if (tsum <= kStageWords) {
                    uint32_t pos = stage_base;
#pragma unroll
                    for (int j = 0; j < K; j++) {
                        base[j] = pos;
                        const int32_t *src = win.times + readlane64(c_off, (uint32_t)j * GT + u);
                        for (uint32_t r = (uint32_t)lane; r < tn[j]; r += kLanes) gs_lds[pos + r] = ld_word(src, r);
                        pos += tn[j];
                    }
                    wave_lds_sync();
                    lstaged = true;
                }
            }
            const int y0 = (int)((g.truth >> state0) & 1);     // zero-delay settled value at t = 0
            int32_t cnt = 0, acc = 0, z = 0, wl = 0;
            // the lane's walk; seed >= 0: an output edge to y0 pending there
            // at t = 0 (continuous segments only)
            auto run = [&](int32_t seed) {
                if (lstaged) {
                    Cursor<K, false, true> P;
#pragma unroll
                    for (int j = 0; j < K; j++) {
                        P.base[j] = base[j];
                        P.idx[j] = lo[j];
                        P.end[j] = hi[j];
                        // with interconnect delays, each staged net list becomes
                        // the pin's arrival list first
                        if (WIRES)
                            wire_filter_lds(base[j], lo[j], P.end[j], (state0 >> j) & 1u, arc.wr[j], arc.wf[j], transport);
                    }
                    P.state = state0;
                    P.transport = transport;
                    walk_lds<K, CAP>(P, arc, g.truth, T, y0, lut_base, out_lane, seed, cnt, wl);
                } else {
                    Cursor<K, WIRES, false> P;
#pragma unroll
                    for (int j = 0; j < K; j++) {
                        P.chunk[j] = win.times + readlane64(c_off, (uint32_t)j * GT + u);
                        P.idx[j] = lo[j];
                        P.end[j] = hi[j];
                    }
                    P.state = state0;
                    P.transport = transport;
                    walk<K, WIRES, false, 0, CAP>(P, arc, g.truth, T, y0, lut_base, out_lane, nullptr, 0, seed, cnt, acc,
                                                  z, wl);
                }
            };
            // Continuous segments: a lane's list keeps the edges before the
            // end of its cycle; the one edge still pending there (at most
            // one, Algorithm 1 cancels a pending edge rather than queueing a
            // second) moves to the next cycle of the segment, which starts
            // with it pending.  Every lane first walks as if nothing were
            // pending; lanes whose carry-in differs are evaluated again until
            // no carry changes.  The carry chain runs upwards through the
            // lanes and each pass settles at least the lowest lane still
            // open, so this ends within 64 passes.
            // A lane with a carry-in W whose first pin event comes no
            // earlier than W evolves as its first walk did, after the
            // pending edge has matured (no event meets it, and the walk's
            // own decisions read the same values), so its list is W followed
            // by that walk's list: it is not walked again (`pre` = W).
            int32_t cin = -1, pre = -1, nlds = 0;
            bool cout_taken = false, cout_pre = false;
            uint32_t p = 0;                                     // the lane's cycle within its segment
            if constexpr (!CONT) {
                run(-1);
                nlds = cnt;
            } else {
                const uint32_t p0 = (tile * kLanes) % seg_len;  // uniform
                p = p0 + (uint32_t)lane;
                if (seg_len >= (uint32_t)kLanes) p = p >= seg_len ? p - seg_len : p;
                else p %= seg_len;
                const bool sstart = p == 0, send = p == seg_len - 1;
                int32_t tfirst = kInf;                          // the lane's first pin event
#pragma unroll
                for (int j = 0; j < K; j++) {
                    if (lo[j] < hi[j]) {
                        const int32_t e = lstaged ? gs_lds[base[j] + lo[j]]
                                                 : ld_word(win.times + readlane64(c_off, (uint32_t)j * GT + u), lo[j]);
                        tfirst = min(tfirst, e);
                    }
                }
                int32_t cnt_s = 0, wl_s = 0, acc_s = 0;         // the first walk
                bool spec = true;                               // LDS slots and acc hold the first walk
                bool walk_now = true;
                int32_t seed = -1, co = -1;
                for (uint32_t pass = 0;; pass++) {
                    if (walk_now) {
                        acc = 0;
                        run(seed);
                        spec = seed < 0;
                    }
                    if (pass == 0) {
                        cnt_s = cnt;
                        wl_s = wl;
                        acc_s = acc;
                    }
                    const int32_t last = cnt > 0 ? wl : pre;
                    co = (active && !send && last >= T) ? last - T : -1;
                    int32_t ni = (int32_t)wave_shr1((uint32_t)(co + 1)) - 1;
                    if (lane == 0) ni = carry;
                    if (sstart || !active) ni = -1;
                    const bool redo = ni != cin;
                    if (__ballot(redo) == 0) break;
                    if (pass > (uint32_t)kLanes) {                  // unreachable (see above): fail the round
                        if (lane == 0)
                            __hip_atomic_fetch_or(glob(win.flags + 3), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    walk_now = false;
                    if (redo) {
                        cin = ni;
                        if (spec && tfirst >= ni) {             // also ni < 0: the first walk stands
                            pre = ni;
                            cnt = cnt_s;
                            wl = wl_s;
                            acc = acc_s;
                        } else {
                            pre = -1;
                            seed = ni;
                            walk_now = true;
                        }
                    }
                }
                carry = __builtin_amdgcn_readlane(co, kLanes - 1);
                nlds = cnt;
                cout_taken = co >= 0;
                if (cout_taken) {
                    if (cnt > 0) cnt--;                         // the walk's last edge leaves
                    else {
                        pre = -1;                               // the carried-in edge passes through
                        cout_pre = true;
                    }
                }
            }
            const int yi = y0 ^ (cin >= 0 ? 1 : 0);         // the output's value at t = 0

            const uint32_t ucnt = (uint32_t)cnt + (pre >= 0 ? 1u : 0u);    // the lane's final list
            const uint32_t incl = wave_incl_scan(ucnt);
            const uint32_t total = (uint32_t)lane63(incl);
            const uint64_t mask = __ballot(active && yi);
            const uint64_t ci = (uint64_t)out_row * ntile + tile;
            bool ok = true;
            if (total > kMaxChunk) {
                if (lane == 0) __hip_atomic_fetch_or(glob(win.flags + 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = false;
            }
            uint64_t obase = 0;
            if (staged) {
                if (used + total > obound) {                    // cannot happen: fail the round, write nothing
                    if (lane == 0)
                        __hip_atomic_fetch_or(glob(win.flags + 3), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                }
                ok = ok && gok;
                obase = ok ? gbase + used : 0;
                if (ok) used += total;
            } else if (ok && total > 0) {
                obase = arena_reserve(win, g.dead, pick, total, lane);
                ok = obase != ~0ull;
                if (!ok) obase = 0;
            }
            st_u16(win.ends + ci * kLanes, (uint32_t)lane,
                   (uint16_t)((ok ? incl : 0u) | ((active && yi) ? 1u << kEndInitShift : 0u)));
            if (lane == 0) {
                ChunkHdr h;
                h.off = ok ? obase : 0;
                h.mask = mask;
                *glob(win.hdr + ci) = h;
            }
            // Copy the staged edges out and sum the lane's T1 terms from its
            // final edge list: each edge toggles the value, and an edge at e
            // to value v adds -min(e, T) if v = 1, +min(e, T) if v = 0.
            int32_t *out_chunk = win.times + obase;
            const uint32_t first = wave_shr1(incl);            // exclusive prefix: the lane's first slot
            int32_t *out = out_chunk + first;
            const int32_t n = cnt < CAP ? cnt : CAP;
            bool walk_acc = !lstaged;                           // acc holds a walk's own sum of its edges
            {
                int v = yi;
                int32_t s1 = 0;
                uint32_t o = first;
                if (CONT && pre >= 0) {                         // the prepended carried-in edge
                    if (ok) st_word(out_chunk, o, pre);
                    o++;
                    v ^= 1;
                    const int32_t ce = min(pre, T);
                    s1 += v ? -ce : ce;
                    if (!lstaged) acc += v ? -ce : ce;          // the first walk's sum lacks it
                }
                for (int32_t i = 0; i < n; i++) {
                    const int32_t e = gs_lds[out_lane + i * kLanes];
                    if (ok) st_word(out_chunk, o + (uint32_t)i, e);
                    v ^= 1;
                    const int32_t ce = min(e, T);
                    s1 += v ? -ce : ce;
                }
                if (lstaged) acc = s1;
            }
            const uint64_t spill = __ballot(nlds > CAP);
            if (spill) {
                // lanes whose list outgrew the staging walk again, from the
                // arena, writing to their place in the output chunk (and
                // returning the complete T1 sum; a carried-in edge is its seed)
                if (nlds > CAP) {
                    Cursor<K, WIRES, false> P;
#pragma unroll
                    for (int j = 0; j < K; j++) {
                        P.chunk[j] = win.times + readlane64(c_off, (uint32_t)j * GT + u);
                        P.idx[j] = lo[j];
                        P.end[j] = hi[j];
                    }
                    P.state = state0;
                    P.transport = transport;
                    int32_t c2, z2, w2;
                    walk<K, WIRES, false, 1, CAP>(P, arc, g.truth, T, y0, lut_base, 0, out, ok ? (int32_t)ucnt : 0,
                                                  cin, c2, acc, z2, w2);
                    walk_acc = true;
                }
                if (lane == 0 && ok)
                    __hip_atomic_fetch_add(glob(win.flags + 2), (unsigned int)__popcll(spill), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            // a walk's sum counted the edge carried out of the cycle (at or
            // after T, so it added -T after a rise and +T after a fall)
            if (CONT && cout_taken && !cout_pre && walk_acc) acc -= ((yi ^ ((ucnt + 1) & 1)) != 0) ? -T : T;
            z = yi ^ (int)(ucnt & 1u);               // every kept edge toggles the output
            tc_sum += total;
            if constexpr (CONT) {
                // a segment's glitch toggles: its edges less the parity of
                // their number, which is its start value XOR its end value
                const uint64_t ms = __ballot(active && p == 0);
                const uint64_t me = __ballot(active && p == seg_len - 1);
                const uint64_t mi = __ballot(yi != 0), mf = __ballot(z != 0);
                uint32_t odd = 0;
                for (uint64_t b = ms | me; b; b &= b - 1) {
                    const int l = __builtin_ctzll(b);
                    if ((ms >> l) & 1u) seg_y = (uint32_t)(mi >> l) & 1u;
                    if ((me >> l) & 1u) odd += seg_y ^ ((uint32_t)(mf >> l) & 1u);
                }
                ig_sum += total - odd;
            } else {
                ig_sum += total - (uint32_t)__popcll(__ballot(cnt & 1));   // a cycle's edges beyond its functional one
            }
            nact_sum += (uint32_t)__popcll(__ballot(active));
            t1_lane += active ? z * T + acc : 0;
#pragma unroll
            for (int j = 0; j < K; j++) {
                if (GT == 4) {
                    ev[j][0] = __builtin_amdgcn_alignbit(ev[j][GT / 2 - 1], ev[j][0], 16);
                    ev[j][GT / 2 - 1] >>= 16;
                } else {
                    ev[j][0] >>= 16;
                }
            }
        }
    }
    const int64_t sum1 = wave_sum64((int64_t)t1_lane);    // up to 64 lanes x 64 tiles x T: beyond 32 bits
    if (lane == 0) {
        __hip_atomic_fetch_add(glob(sg.saif.tc + g.out), (unsigned long long)tc_sum, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (ig_sum)
            __hip_atomic_fetch_add(glob(sg.saif.ig + g.out), (unsigned long long)ig_sum, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(glob(sg.saif.t1 + g.out), (unsigned long long)sum1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(glob(sg.saif.t0 + g.out), (unsigned long long)((int64_t)nact_sum * T - sum1),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Wave w of a launch -> (segment, gate, group of tpw consecutive tiles).
// LDS per wave: 64 words of delay table, the staged fanin words, then either
// (CAP + 1) x 64 staged output words of the per-tile path (the last slot of
// each lane is a spare) or the output stage and lane queue of the compacted
// path.
template <bool WIRES, int CAP, int KMAX, bool REMAP, bool CONT>
__global__ __launch_bounds__(512) void gate_eval_kernel(const Seg *__restrict__ segs, int32_t n_segs, uint64_t n_waves,
                                                        uint32_t tpw)
{
    const int lane = threadIdx.x & (kLanes - 1);
    const uint32_t wpb = blockDim.x / kLanes;
    const uint32_t wib = uniform(threadIdx.x / kLanes);
    const uint64_t w = (uint64_t)blockIdx.x * wpb + wib;
    if (w >= n_waves) return;
    const int si = n_segs == 1 ? 0 : find_seg(segs, n_segs, w);
    // a private copy read through the constant address space: the segment
    // table is never written by the launch, so its fields load with s_load
    // and need not be reloaded after the kernel's own stores
    const Seg sg = *kons(segs + si);
    // a round whose arena or a chunk already overflowed is rerun or failed
    // as a whole: its remaining waves skip their work.  With arena regions
    // (dead nets released) a full region does not stop the round, so that
    // every region that is too small shows up in one try (a chunk that got
    // no space is written empty, which later reads take as no edges).
    if (((sg.win.regions ? 0u : *kons(sg.win.flags)) | *kons(sg.win.flags + 1)) != 0u) return;
    const uint32_t local = (uint32_t)(w - sg.wave_begin);
    const uint32_t ntile = (uint32_t)sg.win.n_tiles;
    const uint32_t ngroup = (ntile + tpw - 1) / tpw;
    const uint32_t gi = local / ngroup;
    const uint32_t grp = local - gi * ngroup;
    const uint32_t tile0 = grp * tpw;
    const uint32_t ntl = min(tpw, ntile - tile0);
    const GateRec g = *kons(sg.gates + sg.gate_begin + gi);
    const uint32_t lut_base = wib * (uint32_t)gate_eval_wave_words(CAP);
    const uint32_t stage_base = lut_base + kLanes;
    const uint32_t out_base = stage_base + kStageWords;
    switch (g.k) {
    case 1: eval_gate<1, WIRES, CAP, REMAP, CONT>(sg, g, tile0, ntl, lane, lut_base, out_base, stage_base); break;
    case 2: eval_gate<2, WIRES, CAP, REMAP, CONT>(sg, g, tile0, ntl, lane, lut_base, out_base, stage_base); break;
    case 3: eval_gate<3, WIRES, CAP, REMAP, CONT>(sg, g, tile0, ntl, lane, lut_base, out_base, stage_base); break;
    case 4: if (KMAX >= 4) eval_gate<(KMAX >= 4 ? 4 : 1), WIRES, CAP, REMAP, CONT>(sg, g, tile0, ntl, lane, lut_base, out_base, stage_base); break;
    case 5: if (KMAX >= 5) eval_gate<(KMAX >= 5 ? 5 : 1), WIRES, CAP, REMAP, CONT>(sg, g, tile0, ntl, lane, lut_base, out_base, stage_base); break;
    case 6: if (KMAX >= 6) eval_gate<(KMAX >= 6 ? 6 : 1), WIRES, CAP, REMAP, CONT>(sg, g, tile0, ntl, lane, lut_base, out_base, stage_base); break;
    default: break;
    }
}

template <bool WIRES, int KMAX, bool REMAP, bool CONT>
static hipError_t launch_ge(const Seg *segs, int32_t n_segs, uint64_t n_waves, int32_t cap, int32_t wpb, uint32_t tpw,
                            hipStream_t s)
{
    const uint64_t blocks = (n_waves + wpb - 1) / wpb;
    const size_t lds = gate_eval_lds_bytes(cap, wpb);
    const dim3 grid((unsigned)blocks), block(kLanes * wpb);
    switch (cap) {
    case 8: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 8, KMAX, REMAP, CONT>), grid, block, lds, s, segs, n_segs, n_waves, tpw); break;
    case 16: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 16, KMAX, REMAP, CONT>), grid, block, lds, s, segs, n_segs, n_waves, tpw); break;
    case 32: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 32, KMAX, REMAP, CONT>), grid, block, lds, s, segs, n_segs, n_waves, tpw); break;
    case 24: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 24, KMAX, REMAP, CONT>), grid, block, lds, s, segs, n_segs, n_waves, tpw); break;
    case 4: hipLaunchKernelGGL((gate_eval_kernel<WIRES, 4, KMAX, REMAP, CONT>), grid, block, lds, s, segs, n_segs, n_waves, tpw); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool REMAP>
static hipError_t launch_ge_r(const Seg *segs, int32_t n_segs, uint64_t n_waves, int32_t wires, int32_t cap,
                              int32_t wpb, int32_t kmax, uint32_t tpw, hipStream_t s)
{
    if (kmax <= 3)
        return wires ? launch_ge<true, 3, REMAP, false>(segs, n_segs, n_waves, cap, wpb, tpw, s)
                     : launch_ge<false, 3, REMAP, false>(segs, n_segs, n_waves, cap, wpb, tpw, s);
    return wires ? launch_ge<true, 6, REMAP, false>(segs, n_segs, n_waves, cap, wpb, tpw, s)
                 : launch_ge<false, 6, REMAP, false>(segs, n_segs, n_waves, cap, wpb, tpw, s);
}

hipError_t launch_gate_eval(const Seg *segs, int32_t n_segs, uint64_t n_waves, int32_t wires, int32_t cap,
                            int32_t wpb, int32_t kmax, uint32_t tpw, int32_t remap, int32_t cont, hipStream_t s)
{
    if (n_waves == 0) return hipSuccess;
    if (wpb < 1 || wpb > 8 || tpw < 1) return hipErrorInvalidValue;
    if (cont) {
        // continuous segments: no interconnect delays, no cone re-simulation
        if (wires || remap) return hipErrorInvalidValue;
        return kmax <= 3 ? launch_ge<false, 3, false, true>(segs, n_segs, n_waves, cap, wpb, tpw, s)
                         : launch_ge<false, 6, false, true>(segs, n_segs, n_waves, cap, wpb, tpw, s);
    }
    return remap ? launch_ge_r<true>(segs, n_segs, n_waves, wires, cap, wpb, kmax, tpw, s)
                 : launch_ge_r<false>(segs, n_segs, n_waves, wires, cap, wpb, kmax, tpw, s);
}

// --------------------------------------------------------------------------
// Delay-edit support: fanout-cone marking (one launch per level, in level
// order, so a gate sees the final marks of every fanin) and clearing of the
// re-simulated nets' SAIF counters.
// --------------------------------------------------------------------------
__global__ void cone_mark_kernel(const GateRec *__restrict__ gates, const PinRec *__restrict__ pins, uint32_t gate_begin,
                                 uint32_t n_gates, uint8_t *mark, unsigned int *count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool in_cone = false;
    if (i < n_gates) {
        const GateRec g = gates[gate_begin + i];
        uint8_t m = mark[g.out];
        for (uint32_t j = 0; j < g.k; j++) m |= mark[pins[g.pin0 + j].net];
        mark[g.out] = m;
        in_cone = m != 0;
    }
    const uint64_t b = __ballot(in_cone);                  // one counter update per wave
    if ((threadIdx.x & (kLanes - 1)) == 0 && b) atomicAdd(count, (unsigned int)__popcll(b));
}

hipError_t launch_cone_mark(const GateRec *gates, const PinRec *pins, uint32_t gate_begin, uint32_t n_gates,
                            uint8_t *mark, unsigned int *count, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(cone_mark_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, gates, pins, gate_begin, n_gates,
                       mark, count);
    return hipGetLastError();
}

__global__ void mark_set_kernel(const uint32_t *__restrict__ nets, uint32_t n, uint8_t *mark)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mark[nets[i]] = 1;
}

hipError_t launch_mark_set(const uint32_t *nets, uint32_t n, uint8_t *mark, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(mark_set_kernel, dim3((n + 255) / 256), dim3(256), 0, s, nets, n, mark);
    return hipGetLastError();
}

// Copies the marked gates (and their pins, at a fixed stride) into a
// level-ordered cone: level l occupies [off[l], off[l+1]); the order inside
// a level follows arrival at the level's cursor (evaluation order inside a
// level does not matter).  slot[out] receives the gate's cone position.
__global__ void cone_place_kernel(const GateRec *__restrict__ gates, const PinRec *__restrict__ pins, uint32_t n_gates,
                                  const uint8_t *__restrict__ mark, const int32_t *__restrict__ level,
                                  const unsigned int *__restrict__ off, unsigned int *cur, GateRec *cg, PinRec *cp,
                                  uint32_t stride, int32_t *slot, uint32_t n_cone)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kLanes - 1);
    GateRec g = {};
    bool in_cone = false;
    int32_t l = 0;
    if (p < n_gates) {
        g = gates[p];
        in_cone = mark[g.out] != 0;
        if (in_cone) l = level[g.out];
    }
    // Gates are in level order, so the cone gates of a wave nearly always
    // share one level: they then take their places with one atomic.
    const uint64_t act = __ballot(in_cone);
    if (!act) return;
    const int first = __builtin_ctzll(act);
    const int32_t l0 = __builtin_amdgcn_readlane(l, first);
    const uint64_t same = __ballot(in_cone && l == l0);
    uint32_t pos = 0;
    if (same == act) {
        uint32_t base = 0;
        if (lane == first) base = atomicAdd(&cur[l0], (unsigned int)__popcll(act));
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, first);
        const uint32_t below = (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
        pos = off[l] + base + below;
    } else if (in_cone) {
        pos = off[l] + atomicAdd(&cur[l], 1u);
    }
    if (!in_cone) return;
    if (pos >= off[l + 1] || pos >= n_cone) return;      // counts and marks disagree: never write outside the cone
    const uint32_t pin0 = g.pin0;
    g.pin0 = pos * stride;
    cg[pos] = g;
    for (uint32_t j = 0; j < g.k; j++) cp[pos * stride + j] = pins[pin0 + j];
    slot[g.out] = (int32_t)pos;
}

hipError_t launch_cone_place(const GateRec *gates, const PinRec *pins, uint32_t n_gates, const uint8_t *mark,
                             const int32_t *level, const unsigned int *off, unsigned int *cur, GateRec *cg, PinRec *cp,
                             uint32_t stride, int32_t *slot, uint32_t n_cone, hipStream_t s)
{
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(cone_place_kernel, dim3((n_gates + 255) / 256), dim3(256), 0, s, gates, pins, n_gates, mark, level,
                       off, cur, cg, cp, stride, slot, n_cone);
    return hipGetLastError();
}

// Per-cycle profile of a finished window: glitch toggles (a lane's edge
// count less its parity) and late nets (the lane's last edge, or its
// arrival through the net's slowest fanout wire for that edge's direction,
// at or after the period), each summed over nets [0, n_nets) per cycle.
// One wave per (64-cycle tile, group of kProfileNets nets), lane = cycle,
// tiles fastest so that neighbouring waves read neighbouring lines of a
// net; a lane's edge count is its inclusive end less its left neighbour's.
// The difference is written as an addition of the shifted negation: a
// subtraction would be fused with the lane shift into a reversed-operand
// form, which gave the negated count on this chip.  One atomic add per
// lane and output.  LATE: also read each lane's last edge (wout: rise and
// fall fanout wire maximum per net, or null for none).
constexpr uint32_t kProfileNets = 2048;

template <bool LATE>
__global__ __launch_bounds__(256) void cycle_profile_kernel(const uint16_t *__restrict__ ends,
                                                            const ChunkHdr *__restrict__ hdr,
                                                            const int32_t *__restrict__ times,
                                                            const int32_t *__restrict__ wout, uint32_t n_nets,
                                                            uint32_t tiles, uint32_t cycles, int32_t T,
                                                            unsigned long long *__restrict__ glitch,
                                                            unsigned long long *__restrict__ late, uint64_t n_waves)
{
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / kLanes) + threadIdx.x / kLanes;
    if (w >= n_waves) return;                                   // whole waves leave together
    const uint32_t lane = threadIdx.x % kLanes;
    // wave-uniform bounds keep the loop scalar, so the unrolled loads below
    // are all in flight before the first wait
    const uint32_t tile = uniform((uint32_t)(w % tiles));
    const uint32_t n0 = uniform((uint32_t)(w / tiles) * kProfileNets);
    const uint32_t n1 = min(n_nets, n0 + kProfileNets);
    const uint64_t stride = (uint64_t)tiles * kLanes;
    const uint16_t *p = ends + ((uint64_t)n0 * tiles + tile) * kLanes;
    uint32_t acc = 0;                                           // at most kProfileNets x kMaxChunk
    uint32_t nlate = 0;
    uint32_t n = n0;
    for (; n + 8 <= n1; n += 8, p += 8 * stride) {
        uint32_t e[8];
#pragma unroll
        for (int u = 0; u < 8; u++) e[u] = ld_u16(p + u * stride, lane);
        uint32_t c[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const uint32_t x = e[u] & kEndCount;
            c[u] = x + wave_shr1(0u - x);
            acc += c[u] - (c[u] & 1u);
        }
        if (LATE) {
            // all eight last-edge reads go out before the first is used
            int32_t last[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const ChunkHdr h = *kons(hdr + (uint64_t)(n + u) * tiles + tile);
                last[u] = 0;
                if (c[u]) last[u] = ld_word(times + h.off, (e[u] & kEndCount) - 1u);
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const uint32_t v_end = ((e[u] >> kEndInitShift) & 1u) ^ (c[u] & 1u);
                const int32_t wr = wout ? *kons(wout + 2 * (uint64_t)(n + u)) : 0;
                const int32_t wf = wout ? *kons(wout + 2 * (uint64_t)(n + u) + 1) : 0;
                nlate += (c[u] && last[u] + (v_end ? wr : wf) >= T) ? 1u : 0u;
            }
        }
    }
    for (; n < n1; n++, p += stride) {
        const uint32_t e = ld_u16(p, lane);
        const uint32_t x = e & kEndCount;
        const uint32_t c = x + wave_shr1(0u - x);
        acc += c - (c & 1u);
        if (LATE && c) {
            const ChunkHdr h = *kons(hdr + (uint64_t)n * tiles + tile);
            const int32_t last = ld_word(times + h.off, x - 1u);
            const uint32_t v_end = ((e >> kEndInitShift) & 1u) ^ (c & 1u);
            const int32_t wr = wout ? *kons(wout + 2 * (uint64_t)n) : 0;
            const int32_t wf = wout ? *kons(wout + 2 * (uint64_t)n + 1) : 0;
            nlate += (last + (v_end ? wr : wf) >= T) ? 1u : 0u;
        }
    }
    const uint32_t cyc = tile * kLanes + lane;
    if (cyc < cycles && glitch && acc)
        __hip_atomic_fetch_add(glob(glitch + cyc), (unsigned long long)acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (LATE && cyc < cycles && nlate)
        __hip_atomic_fetch_add(glob(late + cyc), (unsigned long long)nlate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_cycle_profile(const uint16_t *ends, const ChunkHdr *hdr, const int32_t *times, const int32_t *wout,
                                uint32_t n_nets, uint32_t tiles, uint32_t cycles, int32_t period,
                                unsigned long long *glitch, unsigned long long *late, hipStream_t s)
{
    if (n_nets == 0 || tiles == 0) return hipSuccess;
    const uint64_t n_waves = (uint64_t)((n_nets + kProfileNets - 1) / kProfileNets) * tiles;
    const dim3 grid((unsigned)((n_waves + 3) / 4)), block(256);
    if (late)
        hipLaunchKernelGGL(cycle_profile_kernel<true>, grid, block, 0, s, ends, hdr, times, wout, n_nets, tiles, cycles,
                           period, glitch, late, n_waves);
    else
        hipLaunchKernelGGL(cycle_profile_kernel<false>, grid, block, 0, s, ends, hdr, times, wout, n_nets, tiles,
                           cycles, period, glitch, late, n_waves);
    return hipGetLastError();
}

// Writes edited arc delays into the cone's pin records.
__global__ void edit_apply_kernel(const EditRec *__restrict__ ed, uint32_t n, const int32_t *__restrict__ slot,
                                  PinRec *cp, uint32_t stride, uint32_t n_cone)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const EditRec e = ed[i];
    const int32_t sl = slot[e.out];
    if (sl < 0 || (uint32_t)sl >= n_cone || e.pin >= stride) return;
    PinRec &r = cp[(uint32_t)sl * stride + e.pin];
#pragma unroll
    for (int i = 0; i < 8; i++) r.d[i] = e.d[i];
}

hipError_t launch_edit_apply(const EditRec *ed, uint32_t n, const int32_t *slot, PinRec *cp, uint32_t stride,
                             uint32_t n_cone, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(edit_apply_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ed, n, slot, cp, stride, n_cone);
    return hipGetLastError();
}

__global__ void saif_zero_kernel(const GateRec *__restrict__ gates, uint32_t n, SaifAcc acc)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = gates[i].out;
    acc.tc[o] = 0;
    acc.t0[o] = 0;
    acc.t1[o] = 0;
    acc.ig[o] = 0;
}

hipError_t launch_saif_zero(const GateRec *gates, uint32_t n, SaifAcc acc, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(saif_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, gates, n, acc);
    return hipGetLastError();
}

}  // namespace gs
