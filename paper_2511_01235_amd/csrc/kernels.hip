// gfx950 kernels of the dynamic max-flow path.
//
// Paper map (Kannappan, Kumar, Nasre, "Scalable Maxflow Processing for
// Dynamic Graphs"):
//   k_reset, k_saturate_source     Algorithm 1 initialisation; source
//                                  re-saturation of Algorithm 5
//   k_gr_init, k_gr_level          backward BFS global relabel, Algorithms 4
//                                  and 6 (sink and deficient vertices at 0,
//                                  source pinned at |V|)
//   k_build_worklist               active-vertex worklist (Section 5.2, O1)
//                                  plus the value reduction of Algorithm 5
//   k_pr_{thread,wave,block}       push-relabel kernel, Algorithm 2
//   k_rie_{thread,wave,block}      remove-invalid-edges kernel, Algorithm 3
//   k_batch_*                      update apply and clamp of Algorithm 5
//   k_cut                          cut certificate of Sections 3.1 / 4.3
//
// Every word that bounds a push -- the pusher's own residual res[j] and its
// own excess e(u) -- is read with an agent-scope atomic load, so it is never
// a stale cached copy: only u's worker ever lowers them during a sweep, so the
// amount pushed never exceeds what is there and residuals stay >= 0.  Heights
// of other vertices are plain loads; a stale height only costs extra work (the
// paper's lock-free argument, Section 3.1 note), and the loop stops only after
// a fresh global relabel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdlib>

#include "mf.h"
#include "mf_internal.h"

namespace mf {

namespace {

constexpr int WAVE = 64;
constexpr unsigned long long EMPTY_KEY = ~0ull;

// ---- memory helpers --------------------------------------------------------

__device__ __forceinline__ int32_t ld_res(const int2* cr, int j) {
    return __hip_atomic_load(const_cast<int*>(&cr[j].y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t add_res(int2* cr, int j, int32_t d) {
    return __hip_atomic_fetch_add(&cr[j].y, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t xchg_res(int2* cr, int j, int32_t v) {
    return __hip_atomic_exchange(&cr[j].y, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld_e(const int64_t* e, int v) {
    return __hip_atomic_load(const_cast<int64_t*>(&e[v]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_e(int64_t* e, int v, int64_t d) {
    __hip_atomic_fetch_add(&e[v], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// v receives d > 0; when activations are tracked and v's excess turns
// positive, v goes on the activation list
__device__ __forceinline__ void gain_e(const DevGraph& g, int v, int64_t d) {
    int64_t old = __hip_atomic_fetch_add(&g.e[v], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (g.act && old <= 0 && old + d > 0) {
        int k = atomicAdd(g.act_cnt, 1);
        if (k < g.act_cap) g.act[k] = v;
    }
}
__device__ __forceinline__ void add_bytes(const DevGraph& g, int cls, unsigned long long b) {
    if (g.count_bytes && b)
        atomicAdd(&g.bytes_part[cls * BYTES_SLOTS + (blockIdx.x % BYTES_SLOTS)], b);
}

// A pipelined iteration queued behind the one that ended the loop finds the
// halt word set and leaves every kernel at once.
__device__ __forceinline__ bool halted(const DevGraph& g) { return g.halt && *g.halt; }

// ---- wave primitives ------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Make a value wave-uniform (lane 0's copy) so that every lane takes the same
// branch around the wave collectives below.
__device__ __forceinline__ int bcast(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t bcast64(int64_t x) {
    unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(uint64_t)x);
    unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One DPP step of a 64-lane min over 64-bit keys: each 32-bit half moves
// with the same DPP control; lanes without a valid source keep the identity.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ unsigned long long dpp_min_step(unsigned long long x) {
    unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)(unsigned)x, CTRL,
                                                        ROW_MASK, 0xF, false);
    unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)(unsigned)(x >> 32),
                                                        CTRL, ROW_MASK, 0xF, false);
    unsigned long long y = ((unsigned long long)hi << 32) | lo;
    return y < x ? y : x;
}

// Minimum over the 64 lanes, returned to every lane.  row_shr 1,2,4,8 leaves
// each 16-lane row's running minimum in its lane 15; row_bcast 15 and 31 carry
// rows into the rows above, so lane 63 ends with the wave minimum.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x) {
    x = dpp_min_step<0x111>(x);
    x = dpp_min_step<0x112>(x);
    x = dpp_min_step<0x114>(x);
    x = dpp_min_step<0x118>(x);
    x = dpp_min_step<0x142, 0xA>(x);
    x = dpp_min_step<0x143, 0xC>(x);
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, 63);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ long long wave_sum_i64(long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

// Exclusive prefix sum over the wave; *total gets the wave sum.
__device__ __forceinline__ int wave_excl_scan(int x, int* total) {
    int lane = lane_id();
    int v = x;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int y = __shfl_up(v, d, WAVE);
        if (lane >= d) v += y;
    }
    *total = __shfl(v, WAVE - 1, WAVE);
    return v - x;
}

__device__ __forceinline__ long long wave_excl_scan64(long long x, long long* total) {
    int lane = lane_id();
    long long v = x;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        long long y = __shfl_up(v, d, WAVE);
        if (lane >= d) v += y;
    }
    *total = __shfl(v, WAVE - 1, WAVE);
    return v - x;
}

// Append one item per lane with pred set to list[*counter ...] using one
// atomic per wave (ballot + lane rank).  Must be called by the whole wave.
__device__ __forceinline__ void wave_append(bool pred, int32_t item, int32_t* list, int32_t* counter) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0) return;
    int lane = lane_id();
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader, WAVE);
    if (pred) {
        unsigned long long below = mask & ((1ull << lane) - 1ull);
        list[base + __popcll(below)] = item;
    }
}

template <int BS>
__device__ __forceinline__ long long block_sum_i64(long long x) {
    __shared__ long long part[BS / WAVE];
    x = wave_sum_i64(x);
    int w = threadIdx.x / WAVE;
    if (lane_id() == 0) part[w] = x;
    __syncthreads();
    long long r = 0;
    if (threadIdx.x < WAVE) {
        r = threadIdx.x < BS / WAVE ? part[threadIdx.x] : 0;
        r = wave_sum_i64(r);
    }
    __syncthreads();
    return r;  // valid in wave 0
}

// Which part of the work a block does: block bid of nb.  Ordinary launches
// use the hardware grid; the per-graph solver gives each graph one block
// that does everything (bid 0 of 1).
struct Par {
    int bid, nb;
};
__device__ __forceinline__ Par hw_par() { return Par{(int)blockIdx.x, (int)gridDim.x}; }

// ---- initialisation (Algorithm 1) -----------------------------------------

__global__ void k_fill_i32(int32_t* p, int32_t value, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_reset(DevGraph g, int64_t slot_cap) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < slot_cap; j += stride)
        g.cr[j].y = g.cap[j];
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.n; v += stride) {
        g.e[v] = 0;
        g.h[v] = 0;
    }
}

// Push every unit of residual capacity out of s: x = res(s,u); res(s,u) = 0;
// res(u,s) += x; e(u) += x; e(s) -= x.  From zero flow this is exactly
// Algorithm 1's saturation; after a batch it is Algorithm 5's re-saturation
// written as a delta.
__global__ void __launch_bounds__(256) k_saturate_source(DevGraph g) {
    int beg = g.row_ptr[g.s];
    int len = g.row_len[g.s];
    long long sent = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < len; k += gridDim.x * blockDim.x) {
        int j = beg + k;
        int32_t x = g.cr[j].y;
        if (x > 0) {
            g.cr[j].y = 0;
            add_res(g.cr, g.rev[j], x);
            add_e(g.e, g.cr[j].x, x);
            sent += x;
        }
    }
    long long tot = block_sum_i64<256>(sent);
    if (threadIdx.x == 0 && tot) add_e(g.e, g.s, -tot);
}

// Static push-pull: the sink pulls every residual in-edge w->t full; w may
// turn deficient and is then an extra root of the next relabel.
__global__ void __launch_bounds__(256) k_saturate_sink(DevGraph g) {
    int beg = g.row_ptr[g.t];
    int len = g.row_len[g.t];
    long long got = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < len; k += gridDim.x * blockDim.x) {
        int j = beg + k;            // slot t->w; the in-edge w->t is its reverse
        int w = g.cr[j].x;
        if (w == g.s) continue;     // the source's edges are the source's to saturate
        int r = g.rev[j];
        int32_t x = xchg_res(g.cr, r, 0);
        if (x > 0) {
            add_res(g.cr, j, x);
            add_e(g.e, w, -(int64_t)x);
            got += x;
        }
    }
    long long tot = block_sum_i64<256>(got);
    if (threadIdx.x == 0 && tot) add_e(g.e, g.t, tot);
}

__global__ void __launch_bounds__(256) k_mark_side(DevGraph g, uint8_t* side) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x)
        side[v] = g.h[v] == g.n ? 1 : 0;
}

// Saturate every residual slot from side 1 to side 0 (a slot's owner is the
// column of its reverse slot; free slack slots have no reverse).
__global__ void __launch_bounds__(256) k_saturate_cut(DevGraph g, const uint8_t* side, int64_t slot_cap) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < slot_cap;
         j += (int64_t)gridDim.x * blockDim.x) {
        int2 c = g.cr[j];
        if (c.y <= 0 || side[c.x] != 0) continue;
        int r = g.rev[j];
        if (r < 0) continue;
        int u = g.cr[r].x;
        if (side[u] != 1) continue;
        int32_t x = xchg_res(g.cr, (int)j, 0);
        if (x > 0) {
            add_res(g.cr, r, x);
            add_e(g.e, u, -(int64_t)x);
            add_e(g.e, c.x, (int64_t)x);
        }
    }
}

// ---- global relabel (Algorithms 4 and 6) ----------------------------------

// Zero what one global relabel and the worklist build after it accumulate.
__global__ void k_zero_counters_front(DevCounters* ctr) {
    if (threadIdx.x < 3) {
        ctr->front[threadIdx.x] = 0;
        ctr->unv[threadIdx.x] = 0;
    }
    if (threadIdx.x < 4) ctr->wl[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        ctr->deficit_sum = 0;
        ctr->e_t = 0;
        ctr->bar_count = 0;
        ctr->bar_err = 0;
        ctr->levels = 0;
        ctr->bfs_total = 0;
        ctr->bfs_capped = 0;
        ctr->bfs_raised = 0;
        ctr->bfs_ok = ctr->lab_valid;  // the heights this relabel replaces were a valid labelling
        ctr->lab_valid = 0;
    }
    if (threadIdx.x < 3) {
        ctr->bfs_disc[threadIdx.x] = 0;
        ctr->bfs_cum[threadIdx.x] = 0;
    }
}

// Between push-relabel rounds: clear the worklist counts (before the next
// worklist) or the activation count (before the next push-relabel).
__global__ void k_zero_counts(DevCounters* ctr, int wl, int act, int32_t* bump) {
    if (wl && threadIdx.x < 4) {
        ctr->wl_in[threadIdx.x] = ctr->wl[threadIdx.x];  // the lists the next build reads
        ctr->wl[threadIdx.x] = 0;
    }
    if (act && threadIdx.x == 0) ctr->act = 0;
    if (wl && threadIdx.x == 0) {
        ctr->round_deficit = 0;
        ctr->round_raised = 0;
    }
    if (bump && threadIdx.x == 0) *bump += 1;  // a fresh epoch for the next-worklist marks
}

// End of a pipelined iteration queued behind BFS levels 0..level_end-1: if
// its BFS ended there and its relabel's worklist (set aside in wl_in by the
// next-worklist build) was empty -- or, after_round, the worklist of its
// second round, the active set after the first, with every sink at height 0
// -- the loop is over and every
// kernel of the iteration queued behind this one leaves at once.  The same
// test the host makes on the iteration's counters.
__global__ void k_halt_if_done(const DevCounters* ctr, int level_end, int after_round, int32_t* halt) {
    if (threadIdx.x == 0 && (ctr->front[level_end % 3] & 0xFFFFFFFFull) == 0 &&
        (ctr->wl_in[3] == 0 || (after_round && ctr->wl[3] == 0 && ctr->round_raised == 0)))
        *halt = 1;
}

__global__ void k_set_i32(int32_t* p, int32_t value) {
    if (threadIdx.x == 0) *p = value;
}

// dst[i] = src[i] (src may be pinned host memory mapped for the device)
__global__ void k_copy_i32(int32_t* dst, const int32_t* src, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_set_i64(long long* p, long long value) {
    if (threadIdx.x == 0) *p = value;
}

// Append the frontier entries of the lanes that discovered a vertex:
// ceil(row_len / GR_CHUNK) entries {v, offset} per vertex.  One 64-bit atomic
// per wave both reserves the queue positions (low half) and adds the
// vertices' slot counts to the frontier's slot total (high half).
__device__ __forceinline__ void append_entries(int add, int slots, int v, int2* q,
                                               unsigned long long* counter) {
    int total;
    int off = wave_excl_scan(add, &total);
    if (total == 0) return;
    unsigned long long sl = wave_sum_u64((unsigned long long)slots);
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, (sl << 32) | (unsigned long long)total);
    int b = __shfl((int)(unsigned)(base & 0xFFFFFFFFull), 0, WAVE);
    for (int k = 0; k < add; ++k) q[b + off + k] = make_int2(v, k * GR_CHUNK);
}

// Thread t queues the entries of up to U vertices with one atomic per wave:
// for BFS levels that one workgroup runs alone (no other CU contends for the
// counter, and block_append's barriers would only cost).
template <int U>
__device__ __forceinline__ void wave_append(const int (&vs)[U], const int (&adds)[U], const int (&lens)[U],
                                            int2* q, unsigned long long* counter) {
    int add = 0;
    unsigned long long sl = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        add += adds[k];
        sl += adds[k] > 0 ? (unsigned long long)lens[k] : 0ull;
    }
    int tot;
    const int off = wave_excl_scan(add, &tot);
    const unsigned long long wsl = wave_sum_u64(sl);
    if (tot == 0) return;  // wave-uniform
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, (wsl << 32) | (unsigned)tot);
    int p = __shfl((int)(unsigned)(base & 0xFFFFFFFFull), 0, WAVE) + off;
#pragma unroll
    for (int k = 0; k < U; ++k)
        for (int a = 0; a < adds[k]; ++a) q[p++] = make_int2(vs[k], a * GR_CHUNK);
}

// The same for a whole block with one atomic: thread t queues the entries of
// up to U vertices (vs[k] with adds[k] entries and lens[k] slots).  Every
// level-counter atomic goes to the same address from all CUs and XCDs, so
// one per block instead of one per wave is what keeps levels that discover
// hundreds of thousands of vertices short.  Every thread of the block calls
// it (two barriers); s_agg holds BS / WAVE + 1 words.
template <int BS, int U>
__device__ __forceinline__ void block_append(const int (&vs)[U], const int (&adds)[U], const int (&lens)[U],
                                             int2* q, unsigned long long* counter, unsigned long long* s_agg) {
    int add = 0;
    unsigned long long sl = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        add += adds[k];
        sl += adds[k] > 0 ? (unsigned long long)lens[k] : 0ull;
    }
    int wtot;
    const int off = wave_excl_scan(add, &wtot);
    const unsigned long long wsl = wave_sum_u64(sl);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) s_agg[w] = (wsl << 32) | (unsigned)wtot;
    __syncthreads();
    unsigned long long tot = 0;
    int woff = 0;
#pragma unroll
    for (int i = 0; i < BS / WAVE; ++i) {
        const unsigned long long x = s_agg[i];
        if (i < w) woff += (int)(unsigned)(x & 0xFFFFFFFFull);
        tot += x;
    }
    if (threadIdx.x == 0) s_agg[BS / WAVE] = (tot & 0xFFFFFFFFull) ? atomicAdd(counter, tot) : 0ull;
    __syncthreads();
    int p = (int)(unsigned)(s_agg[BS / WAVE] & 0xFFFFFFFFull) + woff + off;
#pragma unroll
    for (int k = 0; k < U; ++k)
        for (int a = 0; a < adds[k]; ++a) q[p++] = make_int2(vs[k], a * GR_CHUNK);
}

// Visited / frontier bitmaps of a global relabel (one bit per vertex).
__device__ __forceinline__ bool bit_of(const unsigned* bm, int v) { return (bm[v >> 5] >> (v & 31)) & 1u; }
__device__ __forceinline__ void set_bit(unsigned* bm, int v) { atomicOr(&bm[v >> 5], 1u << (v & 31)); }

// h(u) was raised by push-relabel (rounds that track it: DevGraph::relab).
__device__ __forceinline__ void mark_relabel(const DevGraph& g, int u) {
    if (g.relab) set_bit(g.relab, u);
}

// WORDS: the bitmaps are written a whole word at a time (a wave's 64
// vertices are consecutive and 64-aligned: two words per bitmap), so they
// need no clearing beforehand; else single bits are set into cleared maps.
template <bool WORDS = false>
__device__ __forceinline__ void gr_init_body(const Par& P, const DevGraph& g, int2* q0, DevCounters* ctr,
                                             const GrBits& bits, int seed_deficits, int cls = KC_GR) {
    const int N = g.n;
    // capped relabel from a valid labelling: the old heights are kept in
    // h_prev; it must label every vertex with excess below |V| (one at |V|
    // cannot reach a sink while every sink is at height 0), and it may stop
    // early only if no deficient vertex sits above height 0
    const bool cap_ok = g.bfs_cap && ctr->bfs_ok;
    long long excess = 0, raised = 0;
    for (int base = P.bid * blockDim.x; base < N; base += P.nb * blockDim.x) {
        int v = base + threadIdx.x;
        int add = 0, slots = 0;
        bool vis = false, front = false;
        if (v < N && g.side && g.side[v] != g.side_keep) {
            g.h[v] = N;                 // the other side: never labelled by this relabel
            vis = true;
        } else if (v < N) {
            // seed_deficits 1: deficient vertices are extra roots; -1: overflowing ones
            bool extra = false;
            const bool other = v != g.pinned && v != g.s && v != g.t;
            int64_t ev = 0;
            if ((seed_deficits || cap_ok) && other) ev = ld_e(g.e, v);
            if (seed_deficits && other) extra = seed_deficits > 0 ? ev < 0 : ev > 0;
            bool seed = v == g.root || extra;
            if (cap_ok) {
                const int ho = g.h[v];
                g.h_prev[v] = ho;
                if (other && ev > 0 && ho < N) excess++;
                if (other && ev < 0 && ho > 0) raised++;
            }
            g.h[v] = seed ? 0 : N;
            if (seed) {
                slots = g.row_len[v];
                add = (slots + GR_CHUNK - 1) / GR_CHUNK;
            }
            vis = seed || v == g.pinned;  // the pinned vertex is never labelled
            front = seed;
        }
        if (WORDS) {
            const unsigned long long mv = __ballot(vis), mf = __ballot(front);
            const int lane = lane_id();
            const int w = (v >> 5);
            if ((lane & 31) == 0 && w < bits.nwords) {
                const unsigned hv = lane < 32 ? (unsigned)mv : (unsigned)(mv >> 32);
                const unsigned hf = lane < 32 ? (unsigned)mf : (unsigned)(mf >> 32);
                bits.visited[w] = hv;
                bits.fb[w] = hf;
                bits.fb[(size_t)bits.nwords + w] = 0u;
                bits.fb[2 * (size_t)bits.nwords + w] = 0u;
            }
        } else {
            if (vis) set_bit(bits.visited, v);
            if (front) set_bit(bits.fb, v);
        }
        append_entries(add, slots, v, q0, &ctr->front[0]);
    }
    if (cap_ok) {
        const long long x = wave_sum_i64(excess), r = wave_sum_i64(raised);
        if (lane_id() == 0 && x) atomicAdd(&ctr->bfs_total, (int)x);
        if (lane_id() == 0 && r) atomicAdd(&ctr->bfs_raised, (int)r);
    }
    if (P.bid == 0 && threadIdx.x == 0) {
        // slots of every row that may be labelled, the seeds' included
        ctr->unv[2] = (g.nslots ? *g.nslots : (long long)g.used_slots) - g.row_len[g.pinned];
        // per vertex: height, excess; a capped relabel also reads the old
        // height and keeps it in h_prev
        add_bytes(g, cls, (cap_ok ? 20ull : 12ull) * (unsigned long long)N);
    }
}

__global__ void __launch_bounds__(256) k_gr_init(DevGraph g, int2* q0, DevCounters* ctr, GrBits bits,
                                                 int seed_deficits) {
    if (halted(g)) return;
    gr_init_body<true>(hw_par(), g, q0, ctr, bits, seed_deficits, KC_GRS);
}

// One BFS level.  Top-down (small frontier): each block takes 256 frontier
// entries, prefix-sums their slot counts in LDS and lets consecutive threads
// take consecutive slots of the concatenated rows (coalesced, balanced
// across short and long rows); every neighbour v of a level-`lv` vertex u
// that can still be labelled and has the residual needed (backward: v->u,
// i.e. capsum[j] - res[j] > 0 for slot j = u->v; forward: u->v, res[j] > 0)
// gets lv+1 and joins the next frontier.  Bottom-up (frontier above
// n / bu_div entries, bu_div > 0): every unlabelled vertex v scans its own row
// for a neighbour at height lv with the residual needed (backward: res(v->u)
// = res[j] > 0; forward: res(u->v) = capsum[j] - res[j] > 0) and stops at the
// first.  Both produce exactly the BFS levels.  The frontier size is read on
// the device; an empty frontier makes the launch a no-op, so the host may run
// ahead by several levels.

// Top-down slots per thread per round (loads in flight, and one queue atomic
// per block per GR_TD_U * BS slots).
constexpr int GR_TD_U = 4;

// A vertex gets height lv+1: mark it visited and in the next frontier, queue
// its entries, and return its slot count for the direction counters.
// A capped relabel counts the vertices with excess it labels (v gets height
// lv + 1 here), per level.
__device__ __forceinline__ void reached(const DevGraph& g, DevCounters* ctr, int lv, int v) {
    if (g.bfs_cap && v != g.s && v != g.t && ld_e(g.e, v) > 0) atomicAdd(&ctr->bfs_disc[(lv + 1) % 3], 1);
}

// Whether a capped relabel stops before processing level lv: the vertices
// with excess labelled at levels up to lv are all of them.  Reads only counts
// final before level lv began (level lv - 1's cumulative count, the ones
// labelled at lv), so every block decides alike.
__device__ __forceinline__ int excess_labelled(DevCounters* ctr, int lv) {
    // read at L2: a one-workgroup kernel runs many levels without a fresh L1
    const int before = lv > 0 ? __hip_atomic_load(&ctr->bfs_cum[(lv + 2) % 3], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT) : 0;
    return before + __hip_atomic_load(&ctr->bfs_disc[lv % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The count to reach, or INT_MAX (never stop early) unless the relabel began
// from a valid labelling with every deficient vertex at height 0: only then
// are the old heights lower bounds on the new distances, which keeps the
// labelling of a stopped BFS valid (see worklist_body).
__device__ __forceinline__ int excess_total(DevCounters* ctr) {
    const int ok = __hip_atomic_load(&ctr->bfs_ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int raised = __hip_atomic_load(&ctr->bfs_raised, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ok && raised == 0 ? __hip_atomic_load(&ctr->bfs_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : INT_MAX;
}

__device__ __forceinline__ int discover(const DevGraph& g, DevCounters* ctr, const GrBits& bits, int lv, int v,
                                        int* add) {
    set_bit(bits.visited, v);
    set_bit(bits.fb + (size_t)((lv + 1) % 3) * bits.nwords, v);
    reached(g, ctr, lv, v);
    int len = g.row_len[v];
    *add = (len + GR_CHUNK - 1) / GR_CHUNK;
    return len;
}

// The work of one level for a block of BS threads; cnt = the frontier size.
// bu selects bottom-up.  s_bm, when not null, is this block's LDS copy of the
// bitmap the direction needs (visited for top-down, the current frontier for
// bottom-up), replacing the height gather of every scanned slot by a bit test.
// AGG: one frontier-counter atomic per block round (launches of many
// workgroups); else one per wave (a workgroup that runs the level alone).
template <bool FWD, int BS, bool AGG = true>
__device__ __forceinline__ void gr_level_body(const Par& P, const DevGraph& g, int lv, int cnt,
                                              const int2* qin,
                                              int2* qout, DevCounters* ctr, const GrBits& bits,
                                              bool bu, bool bu_lb, bool bu_wide, const unsigned* s_bm,
                                              int cls = KC_GR) {
    __shared__ int s_u[BS];
    __shared__ int s_beg[BS];
    __shared__ int s_pre[BS + 1];
    __shared__ int s_wsum[BS / WAVE];
    __shared__ unsigned long long s_agg[BS / WAVE + 1];
    // exclusive prefix sum of len over the block into s_pre[0..BS], total in s_pre[BS]
    auto block_prefix = [&](int len) {
        int wtot;
        int wex = wave_excl_scan(len, &wtot);
        if (lane_id() == 0) s_wsum[threadIdx.x / WAVE] = wtot;
        __syncthreads();
        int woff = 0, total = 0;
        for (int w = 0; w < BS / WAVE; ++w) {
            if (w < (int)threadIdx.x / WAVE) woff += s_wsum[w];
            total += s_wsum[w];
        }
        s_pre[threadIdx.x] = woff + wex;
        if (threadIdx.x == BS - 1) s_pre[BS] = total;
        __syncthreads();
        return s_pre[BS];
    };
    // last staged entry k with s_pre[k] <= i
    auto owner = [&](int i) {
        int lo = 0, hi = BS;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (s_pre[mid] <= i) lo = mid;
            else hi = mid;
        }
        return lo;
    };
    const int N = g.n;
    unsigned long long* out_cnt = &ctr->front[(lv + 1) % 3];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    unsigned long long scanned = 0, found = 0, exam = 0;
    // is col at height lv (bottom-up)?  The 1-bit-per-vertex bitmaps stay
    // resident in L2, unlike the 4-byte heights.
    const unsigned* cur_fb = bits.fb + (size_t)(lv % 3) * bits.nwords;
    const unsigned* bm_level = s_bm ? s_bm : cur_fb;
    auto at_level = [&](int c) { return bit_of(bm_level, c); };
    const unsigned* bm_seen = s_bm ? s_bm : bits.visited;
    if (bu && bu_lb) {
        // bottom-up, slot-parallel: the block stages BS consecutive vertices,
        // prefix-sums the row lengths of the unlabelled ones and streams
        // their slots with consecutive threads on consecutive slots; a hit
        // flags the row in LDS
        __shared__ int s_hit[BS];
        for (int base = P.bid * BS; base < N; base += P.nb * BS) {
            const int v = base + tid;
            int len = 0;
            if (v < N && !bit_of(bits.visited, v)) {
                len = g.row_len[v];
                s_beg[tid] = g.row_ptr[v];
                exam += 2;
            }
            s_hit[tid] = 0;
            const int total = block_prefix(len);
            for (int b0 = 0; b0 < total; b0 += BS) {
                const int i = b0 + tid;
                if (i < total) {
                    const int k = owner(i);
                    if (!s_hit[k]) {
                        const int j = s_beg[k] + (i - s_pre[k]);
                        const int2 c = g.cr[j];
                        const int32_t r = FWD ? g.capsum[j] - c.y : c.y;
                        if (r > 0 && at_level(c.x)) s_hit[k] = 1;
                        scanned++;
                    }
                }
            }
            __syncthreads();
            int add = 0, slots = 0;
            if (s_hit[tid]) {
                g.h[v] = lv + 1;
                reached(g, ctr, lv, v);
                add = (len + GR_CHUNK - 1) / GR_CHUNK;
                slots = len;
                found++;
            }
            {
                unsigned long long m = __ballot(add > 0);
                unsigned half = lane < 32 ? (unsigned)m : (unsigned)(m >> 32);
                if ((lane & 31) == 0 && half && v < N) {
                    atomicOr(&bits.visited[v >> 5], half);
                    atomicOr(&bits.fb[(size_t)((lv + 1) % 3) * bits.nwords + (v >> 5)], half);
                }
            }
            {
                const int vs[1] = {v}, adds[1] = {add}, lens[1] = {slots};
                if (AGG) block_append<BS, 1>(vs, adds, lens, qout, out_cnt, s_agg);
                else wave_append<1>(vs, adds, lens, qout, out_cnt);
            }
            __syncthreads();  // s_hit / s_pre are restaged next round
        }
    } else if (bu) {
        // bottom-up: threads check up to BU_THREAD_SLOTS slots of their own
        // row (four loads in flight); longer rows without a hit go to a
        // block-local list that the block's waves finish one row at a time
        __shared__ int s_defer[BS];
        __shared__ int s_dhit[BS];
        __shared__ int s_ndefer, s_ndhit;
        for (int base = P.bid * blockDim.x; base < N; base += P.nb * blockDim.x) {
            if (tid == 0) {
                s_ndefer = 0;
                s_ndhit = 0;
            }
            __syncthreads();
            int v = base + tid;
            int add = 0, slots = 0;
            if (v < N && !bit_of(bits.visited, v)) {
                int beg = g.row_ptr[v], len = g.row_len[v];
                int end = beg + min(len, BU_THREAD_SLOTS);
                exam += 2;  // the row bounds
                bool hit = false;
                if (bu_wide) {
                    for (int j = beg; j < end && !hit; j += 8) {
                        int2 c8[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) c8[q] = j + q < end ? g.cr[j + q] : make_int2(0, 0);
                        int32_t r8[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            r8[q] = j + q < end ? (FWD ? g.capsum[j + q] - c8[q].y : c8[q].y) : 0;
#pragma unroll
                        for (int q = 0; q < 8; ++q) hit = hit || (r8[q] > 0 && at_level(c8[q].x));
                        scanned += (unsigned long long)min(8, end - j);
                    }
                } else {
                    for (int j = beg; j < end && !hit; j += 4) {
                        int2 c4[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) c4[q] = j + q < end ? g.cr[j + q] : make_int2(0, 0);
                        int32_t r4[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            r4[q] = j + q < end ? (FWD ? g.capsum[j + q] - c4[q].y : c4[q].y) : 0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) hit = hit || (r4[q] > 0 && at_level(c4[q].x));
                        scanned += (unsigned long long)min(4, end - j);
                    }
                }
                if (hit) {
                    g.h[v] = lv + 1;
                    reached(g, ctr, lv, v);
                    add = (len + GR_CHUNK - 1) / GR_CHUNK;
                    slots = len;
                    found++;
                } else if (len > BU_THREAD_SLOTS) {
                    s_defer[atomicAdd(&s_ndefer, 1)] = v;
                }
            }
            {   // a wave's 64 vertices are consecutive and 64-aligned: two bitmap
                // words, one atomic OR each from lanes 0 and 32
                unsigned long long m = __ballot(add > 0);
                unsigned half = lane < 32 ? (unsigned)m : (unsigned)(m >> 32);
                if ((lane & 31) == 0 && half && v < N) {
                    atomicOr(&bits.visited[v >> 5], half);
                    atomicOr(&bits.fb[(size_t)((lv + 1) % 3) * bits.nwords + (v >> 5)], half);
                }
            }
            {   // block_append's barriers also publish s_defer / s_ndefer
                const int vs[1] = {v}, adds[1] = {add}, lens[1] = {slots};
                if (AGG) block_append<BS, 1>(vs, adds, lens, qout, out_cnt, s_agg);
                else wave_append<1>(vs, adds, lens, qout, out_cnt);
            }
            const int nd = s_ndefer;
            for (int d = tid / WAVE; d < nd; d += BS / WAVE) {
                int w = s_defer[d];
                int beg = g.row_ptr[w] + BU_THREAD_SLOTS, end = g.row_ptr[w] + g.row_len[w];
                bool hit = false;
                for (int b = beg; b < end; b += WAVE) {
                    int j = b + lane;
                    bool my = false;
                    if (j < end) {
                        int2 c = g.cr[j];
                        int32_t r = FWD ? g.capsum[j] - c.y : c.y;
                        my = r > 0 && at_level(c.x);
                    }
                    scanned += (unsigned long long)(j < end);
                    if (__ballot(my)) {
                        hit = true;
                        break;
                    }
                }
                if (hit && lane == 0) {
                    g.h[w] = lv + 1;
                    int addw;
                    discover(g, ctr, bits, lv, w, &addw);
                    s_dhit[atomicAdd(&s_ndhit, 1)] = w;
                    found++;
                }
            }
            __syncthreads();
            {   // the long rows that found a parent, queued by the whole block
                const int nh = s_ndhit;
                int vs[1] = {-1}, adds[1] = {0}, lens[1] = {0};
                if (tid < nh) {
                    vs[0] = s_dhit[tid];
                    lens[0] = g.row_len[vs[0]];
                    adds[0] = (lens[0] + GR_CHUNK - 1) / GR_CHUNK;
                }
                if (AGG) block_append<BS, 1>(vs, adds, lens, qout, out_cnt, s_agg);
                else wave_append<1>(vs, adds, lens, qout, out_cnt);
            }
            __syncthreads();  // s_defer / s_dhit and their counts are reused next round
        }
        exam += (unsigned long long)((N + (int)(P.nb * blockDim.x) - 1) / (int)(P.nb * blockDim.x)) / 8;
    } else {
        // entries per block: spread small frontiers over many blocks, up to
        // BS entries per block for large ones
        const int per = min(BS, max(1, (cnt + P.nb - 1) / P.nb));
        for (int eb = P.bid * per; eb < cnt; eb += P.nb * per) {
            // stage this block's entries and prefix-sum their slot counts
            int idx = eb + tid;
            int len = 0;
            if (tid < per && idx < cnt) {
                int2 ent = qin[idx];
                int rl = g.row_len[ent.x];
                s_u[tid] = ent.x;
                s_beg[tid] = g.row_ptr[ent.x] + ent.y;
                len = min(rl - ent.y, GR_CHUNK);
                exam += 3;
            }
            const int total = block_prefix(len);
            scanned += (unsigned long long)total;  // counted once per block (thread 0 below)
            for (int base = 0; base < total; base += GR_TD_U * BS) {
                int vs[GR_TD_U], adds[GR_TD_U], lens[GR_TD_U];
                int2 cr[GR_TD_U];
                int32_t r[GR_TD_U];
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k) {  // the loads of all U slots first
                    const int i = base + k * BS + tid;
                    cr[k] = make_int2(-1, 0);
                    r[k] = 0;
                    if (i < total) {
                        const int lo = owner(i);
                        const int j = s_beg[lo] + (i - s_pre[lo]);
                        cr[k] = g.cr[j];
                        r[k] = FWD ? cr[k].y : g.capsum[j] - cr[k].y;
                    }
                }
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k) {
                    const int v = cr[k].x;
                    vs[k] = v;
                    adds[k] = 0;
                    lens[k] = 0;
                    // pinned is marked visited at init
                    if (r[k] > 0 && !bit_of(bm_seen, v) && atomicCAS(&g.h[v], N, lv + 1) == N) {
                        lens[k] = discover(g, ctr, bits, lv, v, &adds[k]);
                        found++;
                    }
                }
                if (AGG) block_append<BS, GR_TD_U>(vs, adds, lens, qout, out_cnt, s_agg);
                else wave_append<GR_TD_U>(vs, adds, lens, qout, out_cnt);
            }
            __syncthreads();  // LDS is restaged next round
        }
        if (tid != 0) scanned = 0;
    }
    // per scanned slot: col+res (8), capsum (4), plus h[col] (4) without the
    // LDS bitmap; per staged entry or unlabelled vertex its words; per
    // discovered vertex the CAS, two bitmap words and its queue entry, and
    // with a capped relabel its excess (8)
    unsigned long long per_slot = (s_bm ? 12ull : 16ull) - ((bu && !FWD) ? 4ull : 0ull);
    if (g.count_bytes) {
        const unsigned long long per_found = g.bfs_cap ? 32ull : 24ull;
        unsigned long long b = wave_sum_u64(per_slot * scanned + 4ull * exam + per_found * found);
        if (lane == 0) add_bytes(g, cls, b);
    }
}

// Direction of level lv (Beamer's rule, decided on the device): bottom-up
// when the frontier's slots exceed the unvisited slots / alpha and the
// frontier holds more than n / beta vertices.  Every input was final before
// the level started (the frontier's slots, and the unvisited slots of the
// level before minus the frontier's), so all blocks decide alike; block 0
// records this level's unvisited count for the next one.
__device__ __forceinline__ bool choose_bottom_up(const Par& P, const DevGraph& g, DevCounters* ctr, int lv,
                                                 int cnt, const GrTune& tune) {
    long long fs = (long long)(ctr->front[lv % 3] >> 32);
    long long mu = ctr->unv[(lv + 2) % 3] - fs;
    if (P.bid == 0 && threadIdx.x == 0) ctr->unv[lv % 3] = mu;
    if (tune.bu_alpha <= 0) return false;
    return fs * (long long)tune.bu_alpha > mu && (long long)cnt * tune.bu_beta > (long long)g.n;
}

// One BFS level including its bookkeeping: read the frontier size, clear the
// ring slots of level lv+2, choose the direction, optionally stage the
// bitmap into LDS (s_dyn, when stage_ok), and do the level.  Returns the
// frontier size (0: the BFS is over and nothing was done).
template <bool FWD, int BS, bool AGG = true>
__device__ __forceinline__ int gr_level_step(const Par& P, const DevGraph& g, int lv, const int2* qin,
                                             int2* qout, DevCounters* ctr, const GrBits& bits,
                                             const GrTune& tune, unsigned* s_dyn) {
    // a capped relabel whose earlier levels labelled every vertex with excess
    // stops here: this frontier keeps its height lv, the rest get lv + 1
    // (k_build_worklist), and the BFS reads as over.  (The frontier size
    // first: a launch past the BFS's end leaves after one read.)
    const int front_cnt = bcast((int)(unsigned)(ctr->front[lv % 3] & 0xFFFFFFFFull));
    const int labelled = g.bfs_cap && front_cnt ? bcast(excess_labelled(ctr, lv)) : 0;
    const bool capped = g.bfs_cap && front_cnt && labelled >= bcast(excess_total(ctr));
    const int cnt = capped ? 0 : front_cnt;
    if (P.bid == 0 && threadIdx.x == 0) {
        ctr->front[(lv + 2) % 3] = 0;
        if (g.bfs_cap && front_cnt) {
            ctr->bfs_cum[lv % 3] = labelled;
            ctr->bfs_disc[(lv + 2) % 3] = 0;  // counts the labels of level lv + 2 (set during level lv + 1)
        }
        if (lv == 0) ctr->seed_front = ctr->front[0];
        if (cnt) ctr->levels = lv + 1;  // the BFS's depth so far (levels are launched in order)
        if (capped && (ctr->front[lv % 3] & 0xFFFFFFFFull)) {
            ctr->bfs_capped = lv + 1;  // the height of every vertex not reached
            ctr->front[lv % 3] = 0;
        }
    }
    if (cnt == 0) return 0;
    {   // the bitmap of level lv+2 (input of level lv-1, consumed) starts empty
        unsigned* z = bits.fb + (size_t)((lv + 2) % 3) * bits.nwords;
        for (int i = P.bid * blockDim.x + threadIdx.x; i < bits.nwords; i += P.nb * blockDim.x) z[i] = 0u;
    }
    const bool bu = choose_bottom_up(P, g, ctr, lv, cnt, tune);
    const bool stage = s_dyn && tune.lds && (bu || cnt >= tune.stage_min);
    if (stage) {
        const unsigned* src = bu ? bits.fb + (size_t)(lv % 3) * bits.nwords : bits.visited;
        for (int i = threadIdx.x; i < bits.nwords; i += blockDim.x) s_dyn[i] = src[i];
        __syncthreads();
    }
    gr_level_body<FWD, BS, AGG>(P, g, lv, cnt, qin, qout, ctr, bits, bu, tune.bu_lb != 0, tune.bu_wide != 0,
                           stage ? s_dyn : nullptr);
    return cnt;
}

// Level kernel.  BS = 256 (default): four or more blocks per CU, no LDS
// bitmap.  BS = 1024 with the bitmap staged in LDS: one block per CU.
constexpr int GRL_BLOCK_LDS = 1024;

template <bool FWD, int BS>
__global__ void __launch_bounds__(BS) k_gr_level(DevGraph g, int lv, const int2* qin, int2* qout,
                                                 DevCounters* ctr, GrBits bits, GrTune tune) {
    if (halted(g)) return;
    extern __shared__ unsigned s_dyn[];
    gr_level_step<FWD, BS>(hw_par(), g, lv, qin, qout, ctr, bits, tune, tune.lds ? s_dyn : nullptr);
}

// Thin frontiers (deep BFS, e.g. grids): one workgroup runs top-down levels
// back to back with workgroup barriers only, from level lv0 while each
// frontier covers at most max_slots slots.  It stops at the first empty level
// (the BFS is over) or at a level whose frontier is larger (not processed),
// and leaves in ctr->levels the level to continue from.  The frontier bitmaps
// are not kept up to date here (top-down needs only the visited bitmap); the host
// rebuilds the current one before multi-block levels continue.
constexpr int NARROW_BLOCK = 1024;

template <bool FWD>
__global__ void __launch_bounds__(NARROW_BLOCK) k_gr_narrow(DevGraph g, int lv0, int2* q0, int2* q1,
                                                            DevCounters* ctr, GrBits bits, long long max_slots) {
    __shared__ unsigned long long s_front;
    __shared__ int s_stop;
    const Par P{0, 1};
    int lv = lv0;
    // one thread reads the level's counts and takes the capped relabel's
    // decision (as gr_level_step does); the block follows it
    auto level_counts = [&](int l) {
        if (threadIdx.x == 0) {
            s_front = __hip_atomic_load(&ctr->front[l % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stop = 0;
            if (g.bfs_cap) {
                const int labelled = excess_labelled(ctr, l);
                s_stop = labelled >= excess_total(ctr);
                ctr->bfs_cum[l % 3] = labelled;
                ctr->bfs_disc[(l + 2) % 3] = 0;
            }
        }
    };
    level_counts(lv);
    if (threadIdx.x == 0 && lv == 0) ctr->seed_front = s_front;
    __syncthreads();
    for (; lv <= g.n; ++lv) {
        const int2* qin = (lv & 1) ? q1 : q0;
        int2* qout = (lv & 1) ? q0 : q1;
        const unsigned long long front = s_front;
        const int cnt = (int)(unsigned)(front & 0xFFFFFFFFull);
        // over (empty frontier), or a frontier with too many slots for one
        // workgroup: the multi-block levels take it
        if (cnt == 0 || (long long)(front >> 32) > max_slots) break;
        // a capped relabel that has labelled every vertex with excess stops
        if (s_stop) {
            if (threadIdx.x == 0) {
                ctr->bfs_capped = lv + 1;  // the height of every vertex not reached
                ctr->front[lv % 3] = 0;
            }
            break;
        }
        __syncthreads();  // s_front is rewritten below
        if (threadIdx.x == 0) {
            ctr->front[(lv + 2) % 3] = 0;
            // unvisited slots after this level's frontier, as the direction rule keeps them
            long long fs = (long long)(ctr->front[lv % 3] >> 32);
            ctr->unv[lv % 3] = ctr->unv[(lv + 2) % 3] - fs;
        }
        __syncthreads();
        gr_level_body<FWD, NARROW_BLOCK, false>(P, g, lv, cnt, qin, qout, ctr, bits, false, false, false, nullptr,
                                                KC_GRS);
        __syncthreads();
        level_counts(lv + 1);
        __syncthreads();
    }
    if (threadIdx.x == 0) ctr->levels = lv;
}

// The frontier bitmap of the current level from its queue entries.
__global__ void __launch_bounds__(256) k_mark_frontier(const int2* q, int cnt, unsigned* fb) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) set_bit(fb, q[i].x);
}

// Grid-wide barrier for a cooperative launch (all blocks resident).  Block
// leaders arrive on a counter; the last one resets it and bumps the
// generation the others wait on.  The spin is bounded: past the limit the
// leader flags bar_err and stops waiting, and every block leaves its level
// loop at the next check, so the kernel always ends.
constexpr unsigned GRID_SYNC_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ void grid_sync(DevCounters* ctr) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned gen = __hip_atomic_load(&ctr->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev = __hip_atomic_fetch_add(&ctr->bar_count, 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(&ctr->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctr->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&ctr->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > GRID_SYNC_SPIN_LIMIT) {
                    atomicOr(&ctr->bar_err, 1);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
}

template <int BS>
__device__ __forceinline__ void worklist_body(const Par& P, const DevGraph& g, int32_t* wl0, int32_t* wl1,
                                              int32_t* wl2, DevCounters* ctr, int topology, int sign);

// Mid-size frontiers (deep BFS of grid-like graphs, a few thousand to tens
// of thousands of slots per level): a cooperative launch of a few 1024-thread
// workgroups runs top-down levels back to back, separated by grid barriers
// -- a barrier of a few arrivals costs less than a launch.  Each workgroup
// appends the vertices it labels to a segment of its own ({vertex, first
// slot, slots}: one entry per vertex, whose row bounds are read once, when
// it is labelled) and publishes its segment's counts in a record before the
// barrier; after it, every workgroup reads all the records and so knows the
// level's size, its direction and each segment's place in the level, with no
// shared counter and no other read.  The records are the barrier: each is
// one 64-bit word carrying the level it belongs to, stored with release
// order after the workgroup's appends, and a level starts when every
// workgroup's record of it is there.  From level lv0 while the frontier
// covers at most max_slots slots and the level goes top-down (the direction
// rule of the multi-block levels); at an empty frontier the BFS is over, at a
// capped relabel's stop it ends the same way, and a larger frontier or a
// bottom-up level goes back to the global queue (GR_CHUNK pieces, as the
// multi-block levels read it).  It keeps the visited bitmap, not the frontier
// bitmaps (the host rebuilds the current one), and leaves the level to
// continue from in ctr->levels and the counters the other level kernels read
// (frontier ring, unvisited slots, capped-relabel counts) as they would have.
// Every wait on the barrier is bounded: past the limit bar_err is set and
// every workgroup leaves at the next check.
constexpr int GRM_BLOCK = 1024;
static_assert(MED_MAX_BLOCKS <= WAVE, "one record per lane of a wave");
// A workgroup also keeps the first MED_OWN entries it appends in LDS: when
// every segment of a level fits there and none holds more than about twice
// its share, each workgroup takes its own segment from LDS (no gather of
// the level's entries, no search for their segment).
constexpr int MED_OWN = 1024;

// A segment's record: bits 0..7 the tag of the level it belongs to (1..255,
// the launch's level count modulo 255; 0: not written in this launch), then
// the segment's entries and its vertices with excess (MED_CNT_BITS each) and
// its slots (the rest, saturating: past max_slots the level is handed back
// anyway).  Entries per segment stay below 2^MED_CNT_BITS (MED_MAX_SEG).
constexpr int MED_CNT_BITS = 17;
constexpr int MED_SLOT_BITS = 64 - 8 - 2 * MED_CNT_BITS;
static_assert(MED_MAX_SEG < (1 << MED_CNT_BITS), "segment entries fit a record");

__device__ __forceinline__ unsigned med_tag(int k) { return (unsigned)((k - 1) % 255) + 1u; }

__device__ __forceinline__ unsigned long long med_record(unsigned tag, int cnt, int disc, int slots) {
    const unsigned long long smax = (1ull << MED_SLOT_BITS) - 1;
    const unsigned long long sl = (unsigned long long)slots < smax ? (unsigned long long)slots : smax;
    return (unsigned long long)tag | ((unsigned long long)cnt << 8) | ((unsigned long long)disc << (8 + MED_CNT_BITS)) |
           (sl << (8 + 2 * MED_CNT_BITS));
}

// Publish this workgroup's record once every thread's stores are done
// (release: a workgroup that sees the record sees the segment).
__device__ __forceinline__ void med_publish(unsigned long long* rec, unsigned long long v) {
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(rec, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by the first wave: wait until the records of all nb workgroups in
// `rec` carry `tag`, then return lane b's.  The wait is bounded: past the
// limit bar_err is set and *bad returned true.  A ring's record of level k
// cannot be overwritten (by level k + 2) before every workgroup has read
// it: writing level k + 2 needs every record of level k + 1, which each
// workgroup publishes only after reading level k.
__device__ __forceinline__ unsigned long long med_gather(const unsigned long long* rec, int nb, unsigned tag,
                                                         DevCounters* ctr, bool* bad) {
    const int lane = lane_id();
    unsigned long long v = 0;
    unsigned spins = 0;
    *bad = false;
    for (;;) {
        if (lane < nb) v = __hip_atomic_load(&rec[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool ok = lane >= nb || (unsigned)(v & 0xFFull) == tag;
        if (__all(ok)) break;  // wave-uniform
        __builtin_amdgcn_s_sleep(1);
        if (++spins > GRID_SYNC_SPIN_LIMIT) {
            if (lane == 0) atomicOr(&ctr->bar_err, 1);
            *bad = true;
            break;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return lane < nb ? v : 0ull;
}

template <bool FWD>
__global__ void __launch_bounds__(GRM_BLOCK) k_gr_medium(DevGraph g, int lv0, int2* q0, int2* q1,
                                                         DevCounters* ctr, GrBits bits, GrTune tune,
                                                         long long max_slots, MedQueue mq) {
    const int nb = (int)gridDim.x, bid = (int)blockIdx.x, tid = (int)threadIdx.x, lane = lane_id();
    const int N = g.n;
    const bool cap = g.bfs_cap != 0;
    __shared__ int s_off[MED_MAX_BLOCKS + 1];   // entries of the segments before each one
    __shared__ int s_choff[MED_MAX_BLOCKS + 1]; // GR_CHUNK pieces before each one (hand-back)
    __shared__ int s_slots, s_bad;
    __shared__ int s_cnt_b, s_sl_b, s_disc_b;  // this workgroup's appends in the level
    __shared__ int s_beg[GRM_BLOCK], s_pre[GRM_BLOCK + 1];
    __shared__ int4 s_own[2][MED_OWN];   // the first entries of this workgroup's segment, per ring
    __shared__ int s_own_mode;
    __shared__ int s_wsum[GRM_BLOCK / WAVE];
    __shared__ long long s_mu;
    __shared__ int s_lab, s_total;
    int4* const seg_base = mq.q;
    auto seg = [&](int ring, int b) { return seg_base + ((size_t)ring * nb + b) * mq.seg; };
    // exclusive prefix sum over the workgroup, total in s_pre[GRM_BLOCK]
    auto block_prefix = [&](int x) {
        int wtot;
        const int wex = wave_excl_scan(x, &wtot);
        if (lane == 0) s_wsum[tid / WAVE] = wtot;
        __syncthreads();
        int woff = 0, total = 0;
        for (int w = 0; w < GRM_BLOCK / WAVE; ++w) {
            if (w < tid / WAVE) woff += s_wsum[w];
            total += s_wsum[w];
        }
        s_pre[tid] = woff + wex;
        if (tid == GRM_BLOCK - 1) s_pre[GRM_BLOCK] = total;
        __syncthreads();
        return s_pre[GRM_BLOCK];
    };
    // the incoming frontier (global queue, GR_CHUNK pieces) into segments of ring 0
    int cnt0 = 0;
    if (tid == 0) {
        const unsigned long long f = __hip_atomic_load(&ctr->front[lv0 % 3], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        s_slots = (int)(f >> 32);
        s_cnt_b = (int)(unsigned)(f & 0xFFFFFFFFull);
        s_mu = ctr->unv[(lv0 + 2) % 3];
        s_lab = cap ? excess_labelled(ctr, lv0) : 0;
        s_total = cap ? excess_total(ctr) : INT_MAX;
        if (lv0 == 0 && bid == 0) ctr->seed_front = f;
    }
    __syncthreads();
    cnt0 = s_cnt_b;
    // nothing to do here (the host checks the same): the caller carries on from lv0
    if (cnt0 == 0 || (long long)s_slots > max_slots) {
        if (bid == 0 && tid == 0) ctr->levels = lv0;
        return;
    }
    {
        const int2* qin = (lv0 & 1) ? q1 : q0;
        const int per = (cnt0 + nb - 1) / nb;
        const int k0 = min(cnt0, bid * per), k1 = min(cnt0, bid * per + per);
        int4* out = seg(0, bid);
        int sl = 0;
        for (int k = k0 + tid; k < k1; k += GRM_BLOCK) {
            const int2 ent = qin[k];
            const int len = min(g.row_len[ent.x] - ent.y, GR_CHUNK);
            const int4 e4 = make_int4(ent.x, g.row_ptr[ent.x] + ent.y, len, 0);
            out[k - k0] = e4;
            if (k - k0 < MED_OWN) s_own[0][k - k0] = e4;
            sl += len;
        }
        const int bsl = (int)wave_sum_i64(sl);
        if (tid == 0) s_sl_b = 0;
        __syncthreads();
        if (lane == 0 && bsl) atomicAdd(&s_sl_b, bsl);
        __syncthreads();
        med_publish(&mq.rec[bid], med_record(med_tag(1), k1 - k0, 0, s_sl_b));
    }
    int lv = lv0, ring = 0, mode = 0;
    unsigned long long scanned = 0, found = 0, staged = 0;
    for (;;) {
        // the level's records, one per lane of the first wave (waiting for
        // them is the level barrier): sizes, and where each segment sits
        if (tid < WAVE) {
            bool bad;
            const unsigned long long r = med_gather(mq.rec + (size_t)ring * nb, nb, med_tag(lv - lv0 + 1), ctr, &bad);
            const int rc = (int)((r >> 8) & ((1u << MED_CNT_BITS) - 1));
            const int rd = (int)((r >> (8 + MED_CNT_BITS)) & ((1u << MED_CNT_BITS) - 1));
            const int rs = (int)(r >> (8 + 2 * MED_CNT_BITS));
            int off_tot;
            const int off = wave_excl_scan(rc, &off_tot);
            const int slots = (int)wave_sum_i64(rs), disc = (int)wave_sum_i64(rd);
            int cmax = rc;  // the largest segment
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) cmax = max(cmax, __shfl_xor(cmax, d, WAVE));
            if (tid < nb) s_off[tid] = off;
            if (tid == 0) {
                const int share = (off_tot + nb - 1) / nb;
                s_own_mode = cmax <= MED_OWN && cmax <= 2 * share + 64;
                s_off[nb] = off_tot;
                s_slots = slots;
                s_lab += lv > lv0 ? disc : 0;  // the vertices with excess labelled lv
                s_bad = bad || __hip_atomic_load(&ctr->bar_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        const int cnt = s_off[nb];
        const long long fs = s_slots;
        if (s_bad) {
            mode = 5;
            break;
        }
        // 1: BFS over; 2: capped stop; 3: hand back (too large or bottom-up)
        if (cnt == 0) mode = 1;
        else if (s_lab >= s_total) mode = 2;
        else if (fs > max_slots || lv >= N) mode = 3;
        else if (tune.bu_alpha > 0 && fs * tune.bu_alpha > s_mu - fs && (long long)cnt * tune.bu_beta > (long long)N)
            mode = 3;
        if (mode) break;
        __syncthreads();  // every thread has read s_mu above
        if (tid == 0) {
            s_mu -= fs;  // unvisited slots after this level's frontier
            s_cnt_b = s_sl_b = s_disc_b = 0;
        }
        // this workgroup's entries of the level, BS at a time: its own
        // segment from LDS when the level is balanced, else an equal share
        // of the level's entries from the segments in memory
        const bool own = s_own_mode != 0;
        const int per = (cnt + nb - 1) / nb;
        const int e0 = own ? 0 : min(cnt, bid * per);
        const int e1 = own ? s_off[bid + 1] - s_off[bid] : min(cnt, bid * per + per);
        int4* out = seg(ring ^ 1, bid);
        int4* own_next = s_own[ring ^ 1];
        for (int eb = e0; eb < e1; eb += GRM_BLOCK) {
            const int e = eb + tid;
            int len = 0;
            if (e < e1) {
                int4 ent;
                if (own) {
                    ent = s_own[ring][e];
                } else {
                    int lo = 0, hi = nb;  // the segment holding entry e
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_off[mid] <= e) lo = mid;
                        else hi = mid;
                    }
                    ent = seg(ring, lo)[e - s_off[lo]];
                }
                s_beg[tid] = ent.y;
                len = ent.z;
                staged++;
            }
            const int total = block_prefix(len);
            for (int base = 0; base < total; base += GR_TD_U * GRM_BLOCK) {
                int vs[GR_TD_U];
                int32_t r[GR_TD_U];
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k) {  // the loads of all U slots first
                    const int i = base + k * GRM_BLOCK + tid;
                    vs[k] = -1;
                    r[k] = 0;
                    if (i < total) {
                        int lo = 0, hi = GRM_BLOCK;  // last staged entry with s_pre <= i
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (s_pre[mid] <= i) lo = mid;
                            else hi = mid;
                        }
                        const int j = s_beg[lo] + (i - s_pre[lo]);
                        const int2 c = g.cr[j];
                        vs[k] = c.x;
                        r[k] = FWD ? c.y : g.capsum[j] - c.y;
                        scanned++;
                    }
                }
                bool won[GR_TD_U];
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k) {
                    const int v = vs[k];
                    // the pinned vertex and the other side are marked visited at init
                    won[k] = r[k] > 0 && !bit_of(bits.visited, v) && atomicCAS(&g.h[v], N, lv + 1) == N;
                }
                int rp[GR_TD_U], rl[GR_TD_U];
                bool ex[GR_TD_U];
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k) {
                    const int v = vs[k];
                    rp[k] = 0;
                    rl[k] = 0;
                    ex[k] = false;
                    if (won[k]) {
                        set_bit(bits.visited, v);
                        rp[k] = g.row_ptr[v];
                        rl[k] = g.row_len[v];
                        ex[k] = cap && v != g.s && v != g.t && ld_e(g.e, v) > 0;
                        found++;
                    }
                }
                int add = 0, sl = 0, disc = 0;
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k) {
                    add += rl[k] > 0 ? 1 : 0;  // a vertex without slots needs no entry
                    sl += rl[k];
                    disc += ex[k] ? 1 : 0;
                }
                int atot;
                const int aoff = wave_excl_scan(add, &atot);
                const int wsl = (int)wave_sum_i64(sl), wdisc = (int)wave_sum_i64(disc);
                int abase = 0;
                if (lane == 0) {
                    if (atot) abase = atomicAdd(&s_cnt_b, atot);
                    if (wsl) atomicAdd(&s_sl_b, wsl);
                    if (wdisc) atomicAdd(&s_disc_b, wdisc);
                }
                int p = __shfl(abase, 0, WAVE) + aoff;
#pragma unroll
                for (int k = 0; k < GR_TD_U; ++k)
                    if (rl[k] > 0) {
                        const int4 e4 = make_int4(vs[k], rp[k], rl[k], 0);
                        out[p] = e4;
                        if (p < MED_OWN) own_next[p] = e4;
                        ++p;
                    }
            }
            __syncthreads();  // s_beg / s_pre are restaged next round
        }
        __syncthreads();
        med_publish(&mq.rec[(size_t)(ring ^ 1) * nb + bid], med_record(med_tag(lv - lv0 + 2), s_cnt_b, s_disc_b, s_sl_b));
        ++lv;
        ring ^= 1;
    }
    if (mode == 3) {
        // hand the level's frontier back to the global queue in GR_CHUNK
        // pieces: each workgroup counts its segment's pieces and publishes
        // the count (a third ring of records); its own go after the pieces
        // of the segments before it
        int2* qout = (lv & 1) ? q1 : q0;
        const int4* in = seg(ring, bid);
        const int nmine = s_off[bid + 1] - s_off[bid];
        int mine = 0;
        for (int e = tid; e < nmine; e += GRM_BLOCK) mine += (in[e].z + GR_CHUNK - 1) / GR_CHUNK;
        const int wmine = (int)wave_sum_i64(mine);
        if (tid == 0) s_cnt_b = 0;
        __syncthreads();
        if (lane == 0 && wmine) atomicAdd(&s_cnt_b, wmine);
        __syncthreads();
        med_publish(&mq.rec[(size_t)2 * nb + bid], (unsigned long long)s_cnt_b << 8 | 1ull);
        if (tid < WAVE) {
            bool bad;
            const unsigned long long r = med_gather(mq.rec + (size_t)2 * nb, nb, 1u, ctr, &bad);
            int tot;
            const int off = wave_excl_scan((int)(r >> 8), &tot);
            if (tid < nb) s_choff[tid] = off;
            if (tid == 0) s_choff[nb] = tot;
        }
        __syncthreads();
        int pos = s_choff[bid];
        for (int eb = 0; eb < nmine; eb += GRM_BLOCK) {
            const int e = eb + tid;
            int4 ent = make_int4(0, 0, 0, 0);
            int pieces = 0;
            if (e < nmine) {
                ent = in[e];
                pieces = (ent.z + GR_CHUNK - 1) / GR_CHUNK;
            }
            const int tot = block_prefix(pieces);
            const int at = pos + s_pre[tid];
            // an entry read from the global queue at entry is one piece at its
            // own offset; one labelled here starts at its row's first slot
            const int first = e < nmine ? ent.y - g.row_ptr[ent.x] : 0;
            for (int a = 0; a < pieces; ++a) qout[at + a] = make_int2(ent.x, first + a * GR_CHUNK);
            pos += tot;
            __syncthreads();
        }
    }
    if (bid == 0 && tid == 0) {
        const bool over = mode == 1 || mode == 2;
        ctr->front[lv % 3] = over ? 0ull : (((unsigned long long)s_slots << 32) | (unsigned)s_choff[nb]);
        ctr->front[(lv + 1) % 3] = 0;
        ctr->front[(lv + 2) % 3] = 0;
        if (mode == 2) ctr->bfs_capped = lv + 1;  // the height of every vertex not reached (or more)
        ctr->unv[(lv + 2) % 3] = s_mu;
        if (cap && lv > lv0) {  // the labelled count at level lv, as excess_labelled reads it
            ctr->bfs_cum[(lv + 2) % 3] = s_lab;
            ctr->bfs_disc[lv % 3] = 0;
            ctr->bfs_disc[(lv + 1) % 3] = 0;
        }
        ctr->levels = lv;
    }
    if (g.count_bytes) {
        // per scanned slot: col+res (8), capsum (4), the visited word (4);
        // per staged entry its 16 bytes; per labelled vertex the CAS, its row
        // bounds, excess, bitmap word and entry
        const unsigned long long b = wave_sum_u64(16ull * scanned + 16ull * staged + 40ull * found);
        if (lane == 0) add_bytes(g, KC_GRS, b);
    }
}

// Global relabel and worklist build in one cooperative launch: seeds, then
// one level after another separated by grid barriers (same level work as
// k_gr_level), then the worklist and value over the fresh heights.
constexpr int GRP_BLOCK = 1024;

template <bool FWD>
__global__ void __launch_bounds__(GRP_BLOCK) k_gr_persistent(DevGraph g, int2* q0, int2* q1,
                                                             DevCounters* ctr, GrBits bits, GrTune tune,
                                                             int seed_deficits, int32_t* wl0,
                                                             int32_t* wl1, int32_t* wl2,
                                                             int topology, int sign) {
    __shared__ int s_flag[2];
    gr_init_body(hw_par(), g, q0, ctr, bits, seed_deficits);
    grid_sync(ctr);
    int lv = 0;
    for (;; ++lv) {
        // one read per block so that every wave takes the same branch
        if (threadIdx.x == 0) {
            s_flag[0] = (int)(unsigned)(__hip_atomic_load(&ctr->front[lv % 3], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) & 0xFFFFFFFFull);
            s_flag[1] = __hip_atomic_load(&ctr->bar_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int cnt = s_flag[0], bad = s_flag[1];
        if (cnt == 0 || bad) break;
        if (lv > g.n) {  // a BFS has at most n levels
            if (threadIdx.x == 0) atomicOr(&ctr->bar_err, 2);
            break;
        }
        gr_level_step<FWD, GRP_BLOCK>(hw_par(), g, lv, (lv & 1) ? q1 : q0, (lv & 1) ? q0 : q1, ctr, bits,
                                      tune, nullptr);
        grid_sync(ctr);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->levels = lv;
    worklist_body<GRP_BLOCK>(hw_par(), g, wl0, wl1, wl2, ctr, topology, sign);
}

// ---- worklist (Section 5.2, O1) and value (Algorithm 5) --------------------

// sign = +1: active = positive excess below |V| (the solve); sign = -1:
// active = negative excess below |V| (deficits to fill from t).
template <int BS>
__device__ __forceinline__ void worklist_body(const Par& P, const DevGraph& g, int32_t* wl0, int32_t* wl1,
                                              int32_t* wl2, DevCounters* ctr, int topology, int sign) {
    const int N = g.n;
    long long deficit = 0;
    // after a capped relabel that stopped before level L, a vertex it did not
    // reach gets max(L + 1, its old height).  That is a valid labelling: a
    // residual slot between two such vertices keeps h(a) <= h(b) + 1 (it
    // held for the old heights); from such a vertex a to a labelled b, b is
    // at L (a level below L would have reached a) and the old h(a) <= old
    // h(b) + 1 <= L + 1, the old heights being lower bounds on distances.
    // Vertices at |V| stay there.
    const int cap_h = g.bfs_cap ? ctr->bfs_capped : 0;
    for (int base = P.bid * blockDim.x; base < N; base += P.nb * blockDim.x) {
        int v = base + threadIdx.x;
        bool act = false, list = false;
        int len = 0;
        if (v < N) {
            int64_t ev = g.e[v];
            int hv = g.h[v];
            if (cap_h && hv == N && v != g.pinned) {
                hv = max(cap_h, g.h_prev[v]);
                g.h[v] = hv;
            }
            bool other = v != g.s && v != g.t;
            act = other && (sign > 0 ? ev > 0 : ev < 0) && hv < N;
            if (other && ev < 0) deficit += ev;
            if (v == g.t) ctr->e_t = ev;
            len = g.row_len[v];
            list = topology ? (other && len > 0) : act;
        }
        unsigned long long am = __ballot(act);
        if (lane_id() == 0 && am) atomicAdd(&ctr->wl[3], __popcll(am));
        int bin = len <= g.bin0_max ? 0 : (len <= g.bin1_max ? 1 : 2);
        wave_append(list && bin == 0, v, wl0, &ctr->wl[0]);
        wave_append(list && bin == 1, v, wl1, &ctr->wl[1]);
        wave_append(list && bin == 2, v, wl2, &ctr->wl[2]);
    }
    long long tot = block_sum_i64<BS>(deficit);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long*)&ctr->deficit_sum, (unsigned long long)tot);
    if (P.bid == 0 && threadIdx.x == 0) add_bytes(g, KC_WL, 16ull * (unsigned long long)N);
}

__global__ void __launch_bounds__(256) k_build_worklist(DevGraph g, int32_t* wl0, int32_t* wl1,
                                                        int32_t* wl2, DevCounters* ctr,
                                                        int topology, int sign, int guard_level) {
    if (halted(g)) return;
    // The first round's activations start here -- also when the build is
    // skipped below, so that nothing queued behind it finds work: neither
    // the rounds (worklist sizes zero) nor the next-worklist build after the
    // first of them (no activations either).
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->act = 0;
    // guard_level >= 0: queued behind BFS levels up to guard_level - 1 before
    // the host knew whether the BFS ends there; a frontier still waiting at
    // guard_level means it did not, and this build is skipped
    if (guard_level >= 0 && (ctr->front[guard_level % 3] & 0xFFFFFFFFull) != 0) return;
    // the heights are a valid labelling from here until the next relabel
    // starts (push-relabel rounds with remove-invalid-edges keep it so)
    if (g.bfs_cap && blockIdx.x == 0 && threadIdx.x == 0) ctr->lab_valid = 1;
    if (g.relab) {  // the rounds after this build start with no vertex marked as raised
        const int nw = (g.n + 31) >> 5;
        for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) g.relab[w] = 0u;
    }
    worklist_body<256>(hw_par(), g, wl0, wl1, wl2, ctr, topology, sign);
}

// ---- push-relabel (Algorithm 2) --------------------------------------------
//
// Per cycle: if u is active, find its lowest residual neighbour v^ (first slot
// in row order among equal heights), then push d = min(e(u), res(u,v^)) if
// h(u) > h^ with four atomics, else lift h(u) = h^ + 1 (capped at |V|).  The
// scan compares the height it read once (the note after Section 3.1's
// termination proof).  A row with no residual slot lifts u to |V|.

// PULL = false: u pushes along its residual out-slot j (res[j]) and
// "amount" is its excess.  PULL = true (filling a deficit from t, the
// mirror image used to complete a preflow): u pulls along the residual of
// the in-edge col->u (res[rev[j]]) and "amount" is minus its excess.
template <bool PULL>
__device__ __forceinline__ int32_t scan_res(const DevGraph& g, int j) {
    return PULL ? ld_res(g.cr, g.rev[j]) : ld_res(g.cr, j);
}

template <bool PULL>
__device__ __forceinline__ int64_t amount(const DevGraph& g, int u) {
    int64_t e = ld_e(g.e, u);
    return PULL ? -e : e;
}

template <bool PULL>
__device__ __forceinline__ void do_push(DevGraph& g, int u, int j, int64_t eu) {
    int jo = PULL ? g.rev[j] : j;  // residual that shrinks
    int ji = PULL ? j : g.rev[j];  // residual that grows
    int32_t r = ld_res(g.cr, jo);
    int64_t d = eu < (int64_t)r ? eu : (int64_t)r;
    if (d <= 0) return;
    add_res(g.cr, jo, -(int32_t)d);
    add_res(g.cr, ji, (int32_t)d);
    int w = g.cr[j].x;
    add_e(g.e, PULL ? w : u, -d);
    if (PULL) add_e(g.e, u, d);
    else gain_e(g, w, d);
}

// Move d along slot j of u without touching e(u) (the caller settles u's
// excess once for all the moves of a cycle): the residual the move uses
// shrinks, its reverse grows, and the neighbour's excess changes by d.
template <bool PULL>
__device__ __forceinline__ void move_along(DevGraph& g, int j, int32_t d) {
    int jo = PULL ? g.rev[j] : j;
    int ji = PULL ? j : g.rev[j];
    add_res(g.cr, jo, -d);
    add_res(g.cr, ji, d);
    if (PULL) add_e(g.e, g.cr[j].x, -(int64_t)d);
    else gain_e(g, g.cr[j].x, d);
}

// Key of slot j for the lowest-neighbour search: (h(col) << 32 | j) when the
// residual the move would use is positive, else ~0.  The slot's col and res
// come from one coherent 64-bit load.
__device__ __forceinline__ unsigned long long ld_slot(const int2* cr, int j) {
    return __hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<int2*>(&cr[j])),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Scan slots [b + 0, b + STEP, ... b + (U-1)*STEP] (those below end) and fold
// their keys into best.  All loads of the group are issued before any height
// gather, so U slots are in flight per lane.
template <bool PULL, int U, int STEP>
__device__ __forceinline__ void scan_group(const DevGraph& g, int b, int end, unsigned long long& best) {
    unsigned long long sv[U];
    int32_t r[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        int j = b + q * STEP;
        sv[q] = j < end ? ld_slot(g.cr, j) : 0ull;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
        int j = b + q * STEP;
        r[q] = j < end ? (PULL ? ld_res(g.cr, g.rev[j]) : (int32_t)(sv[q] >> 32)) : 0;
    }
    unsigned hv[U];
#pragma unroll
    for (int q = 0; q < U; ++q) hv[q] = r[q] > 0 ? (unsigned)g.h[(int)(unsigned)sv[q]] : 0u;
#pragma unroll
    for (int q = 0; q < U; ++q) {
        int j = b + q * STEP;
        if (r[q] > 0) {
            unsigned long long key = ((unsigned long long)hv[q] << 32) | (unsigned)j;
            if (key < best) best = key;
        }
    }
}

constexpr int PR_UNROLL = 4;
// Rows above the wave bin: loads in flight per lane.  Four keep the kernel
// within 64 VGPRs, so that two 1024-thread workgroups fit a CU (eight: 80
// VGPRs and one workgroup per CU; rmat20 repairs 1.26 -> 1.20 ms).
constexpr int PR_UNROLL_BLOCK = 4;

// Per-vertex bodies of Algorithm 2; each returns the algorithmic bytes it
// moved.  A relabel is followed by the push of the next cycle on the same
// scan (the lowest neighbour it found is now admissible), two of the KC
// cycles for one scan of the row.  A push goes to the lowest neighbour the
// scan found and then on to every other residual slot whose neighbour is
// still at that height, until the excess is gone: the cycles Algorithm 2
// would spend saturating one lowest neighbour after another under the same
// heights, done in one pass (heights only rise during push-relabel, so a
// neighbour still at the scanned minimum is still admissible).  Thread: one lane owns u.  Wave: u is wave-uniform.  Block: u is
// block-uniform and the whole block scans its row.
template <bool PULL>
__device__ __forceinline__ unsigned long long pr_thread_item(DevGraph& g, int u, int kc) {
    const int N = g.n;
    int beg = g.row_ptr[u];
    int end = beg + g.row_len[u];
    int hu = g.h[u];
    unsigned long long bytes = 16;
    for (int c = 0; c < kc && hu < N; ++c) {
        int64_t eu = amount<PULL>(g, u);
        if (eu <= 0) continue;
        unsigned long long best = ~0ull;
        for (int b = beg; b < end; b += PR_UNROLL) scan_group<PULL, PR_UNROLL, 1>(g, b, end, best);
        bytes += 12ull * (unsigned long long)(end - beg);
        if (best == ~0ull) {
            hu = N;
            g.h[u] = N;
            mark_relabel(g, u);
            break;
        }
        int bh = (int)(best >> 32);
        int bj = (int)(unsigned)best;
        if (hu <= bh) {
            hu = bh + 1 < N ? bh + 1 : N;
            g.h[u] = hu;
            mark_relabel(g, u);
            bytes += 4;
            if (hu >= N || ++c >= kc) break;
        }
        // push to bj, then to the following slots still at height bh, in
        // slot order, until the excess is gone
        int64_t left = eu;
        for (int j = bj; j < end && left > 0; ++j) {
            int32_t r = scan_res<PULL>(g, j);
            if (r <= 0 || (j != bj && g.h[g.cr[j].x] != bh)) continue;
            int32_t d = left < (int64_t)r ? (int32_t)left : r;
            move_along<PULL>(g, j, d);
            left -= d;
            bytes += 48;
        }
        if (left != eu) add_e(g.e, u, PULL ? eu - left : left - eu);
        bytes += 12ull * (unsigned long long)(end - bj);
    }
    return bytes;
}

template <bool PULL>
__device__ __forceinline__ unsigned long long pr_wave_item(DevGraph& g, int u, int kc) {
    const int N = g.n;
    const int lane = lane_id();
    int beg = bcast(g.row_ptr[u]);
    int end = beg + bcast(g.row_len[u]);
    int hu = bcast(g.h[u]);
    // wave-uniform terms on lane 0, per-lane terms on each lane: the caller
    // sums the wave
    unsigned long long bytes = lane == 0 ? 16 : 0;
    for (int c = 0; c < kc && hu < N; ++c) {
        int64_t eu = bcast64(amount<PULL>(g, u));
        if (eu <= 0) continue;
        unsigned long long best = ~0ull;
        for (int b = beg; b < end; b += PR_UNROLL * WAVE)
            scan_group<PULL, PR_UNROLL, WAVE>(g, b + lane, end, best);
        best = wave_min_u64(best);
        if (lane == 0) bytes += 12ull * (unsigned long long)(end - beg);
        if (best == ~0ull) {
            hu = N;
            if (lane == 0) {
                g.h[u] = N;
                mark_relabel(g, u);
            }
            break;
        }
        int bh = (int)(best >> 32);
        int bj = (int)(unsigned)best;
        if (hu <= bh) {
            hu = bh + 1 < N ? bh + 1 : N;
            if (lane == 0) {
                g.h[u] = hu;
                mark_relabel(g, u);
                bytes += 4;
            }
            if (hu >= N || ++c >= kc) break;
        }
        // push to bj, then to the following slots still at height bh, in
        // slot order (a wave prefix sum hands out the excess), until the
        // excess is gone
        int64_t left = eu;
        for (int b = bj; b < end && left > 0; b += WAVE) {
            int j = b + lane;
            int32_t r = j < end ? scan_res<PULL>(g, j) : 0;
            bool cand = r > 0 && (j == bj || g.h[g.cr[j].x] == bh);
            long long tot;
            long long ex = wave_excl_scan64(cand ? (long long)r : 0ll, &tot);
            if (cand && ex < left) {
                int64_t room = left - ex;
                move_along<PULL>(g, j, room < (int64_t)r ? (int32_t)room : r);
                bytes += 48;
            }
            left -= tot < left ? tot : left;
            bytes += 12ull * (unsigned long long)(j < end);
        }
        if (lane == 0 && left != eu) add_e(g.e, u, PULL ? eu - left : left - eu);
    }
    return bytes;
}

template <bool PULL, int BS>
__device__ __forceinline__ unsigned long long pr_block_item(DevGraph& g, int u, int kc) {
    // Long rows: one pass per cycle.  While it looks for the lowest
    // neighbour, the pass already pushes to every residual slot whose
    // neighbour is at h(u) - 1 -- under a valid labelling the lowest height a
    // neighbour can have, so these are the pushes Algorithm 2's next cycles
    // would make -- until the excess is gone.  Excess left over: the minimum
    // of the pass decides as in Algorithm 2 (relabel to it + 1, or a push to
    // a lower slot left by stale heights).
    __shared__ unsigned long long part[BS / WAVE];
    __shared__ int64_t e_sh;
    __shared__ unsigned long long taken;   // excess handed out by the current pass
    const int N = g.n;
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    int beg = g.row_ptr[u];
    int end = beg + g.row_len[u];
    int hu = g.h[u];
    // block-uniform terms on thread 0, per-thread terms on each thread: the
    // caller sums the block
    unsigned long long bytes = threadIdx.x == 0 ? 16 : 0;
    for (int c = 0; c < kc && hu < N; ++c) {
        if (threadIdx.x == 0) {
            e_sh = amount<PULL>(g, u);
            taken = 0ull;
        }
        __syncthreads();
        const int64_t eu = e_sh;
        __syncthreads();
        if (eu <= 0) continue;
        const unsigned target = (unsigned)(hu - 1);
        unsigned long long best = ~0ull;
        bool done = false;
        for (int b0 = beg; b0 < end && !done; b0 += PR_UNROLL_BLOCK * BS) {
            const int b = b0 + threadIdx.x;
            unsigned long long sv[PR_UNROLL_BLOCK];
#pragma unroll
            for (int q = 0; q < PR_UNROLL_BLOCK; ++q) {
                int j = b + q * BS;
                sv[q] = j < end ? ld_slot(g.cr, j) : 0ull;
            }
            int32_t r[PR_UNROLL_BLOCK];
#pragma unroll
            for (int q = 0; q < PR_UNROLL_BLOCK; ++q) {
                int j = b + q * BS;
                r[q] = j < end ? (PULL ? ld_res(g.cr, g.rev[j]) : (int32_t)(sv[q] >> 32)) : 0;
            }
            unsigned hv[PR_UNROLL_BLOCK];
#pragma unroll
            for (int q = 0; q < PR_UNROLL_BLOCK; ++q) hv[q] = r[q] > 0 ? (unsigned)g.h[(int)(unsigned)sv[q]] : 0u;
#pragma unroll
            for (int q = 0; q < PR_UNROLL_BLOCK; ++q) {
                const int j = b + q * BS;
                const bool cand = r[q] > 0 && hv[q] == target;
                if (r[q] > 0) {
                    unsigned long long key = ((unsigned long long)hv[q] << 32) | (unsigned)j;
                    if (key < best) best = key;
                }
                long long tot;
                long long ex = wave_excl_scan64(cand ? (long long)r[q] : 0ll, &tot);
                if (tot == 0) continue;  // wave-uniform
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&taken, (unsigned long long)tot);
                const int64_t before = (int64_t)bcast64((long long)base) + ex;
                if (cand && before < eu) {
                    int64_t room = eu - before;
                    move_along<PULL>(g, j, room < (int64_t)r[q] ? (int32_t)room : r[q]);
                    bytes += 48;
                }
            }
#pragma unroll
            for (int q = 0; q < PR_UNROLL_BLOCK; ++q) bytes += b + q * BS < end ? 12ull : 0ull;
            done = (int64_t)bcast64((long long)taken) >= eu;  // wave-uniform: this wave stops
        }
        best = wave_min_u64(best);
        if (lane == 0) part[wv] = best;
        __syncthreads();
        unsigned long long x = lane < BS / WAVE ? part[lane] : ~0ull;
        best = wave_min_u64(x);  // every wave computes the same block minimum
        const int64_t moved = (int64_t)taken < eu ? (int64_t)taken : eu;
        __syncthreads();
        if (threadIdx.x == 0 && moved) add_e(g.e, u, PULL ? moved : -moved);
        if (moved >= eu) continue;  // the excess is gone (more may arrive)
        // excess left: the scan saw the whole row
        if (best == ~0ull) {
            hu = N;
            if (threadIdx.x == 0) {
                g.h[u] = N;
                mark_relabel(g, u);
            }
            break;
        }
        const int bh = (int)(best >> 32);
        const int bj = (int)(unsigned)best;
        if (bh < hu - 1) {
            // a neighbour below h(u) - 1 (heights moved meanwhile): push there
            if (threadIdx.x == 0) {
                do_push<PULL>(g, u, bj, eu - moved);
                bytes += 48;
            }
        } else if (bh >= hu) {
            hu = bh + 1 < N ? bh + 1 : N;
            if (threadIdx.x == 0) {
                g.h[u] = hu;
                mark_relabel(g, u);
                bytes += 4;
            }
        }
        // bh == hu - 1: those slots were saturated by this pass; the next pass rescans
    }
    __syncthreads();  // part / e_sh / taken are reused by the next item
    return bytes;
}

template <bool PULL>
__global__ void __launch_bounds__(BLOCK_PR, 8) k_pr_block(DevGraph g, const int32_t* wl, int count,
                                                       int kc, DevCounters* ctr, const int32_t* dcount) {
    if (halted(g)) return;
    (void)ctr;
    const int cnt = dcount ? *dcount : count;
    unsigned long long bytes = 0;
    for (int it = blockIdx.x; it < cnt; it += gridDim.x)  // whole blocks
        bytes += pr_block_item<PULL, BLOCK_PR>(g, wl[it], kc);
    if (g.count_bytes) {
        const unsigned long long b = wave_sum_u64(bytes);
        if (lane_id() == 0 && b) add_bytes(g, KC_PR, b);
    }
}

// One launch for a round's thread and wave bins (the workgroup bin has its
// own 1024-thread launch: in one kernel with these its registers would halve
// their occupancy).  The 256-thread workgroups take virtual blocks in turn:
// first BS / WAVE rows of the wave bin per block, then BS rows of the thread
// bin.  Bin sizes: dcount[0..1] on the device when dcount is set, else c0, c1.
struct BinSizes {
    int c0, c1, c2;
};
__device__ __forceinline__ BinSizes bin_sizes(const int32_t* dcount, int c0, int c1, int c2) {
    if (dcount) return BinSizes{dcount[0], dcount[1], dcount[2]};
    return BinSizes{c0, c1, c2};
}

constexpr int PR_SMALL_BLOCK = 256;

template <bool PULL>
__global__ void __launch_bounds__(PR_SMALL_BLOCK) k_pr_small(DevGraph g, const int32_t* wl0, const int32_t* wl1,
                                                             int c0, int c1, int kc, const int32_t* dcount) {
    if (halted(g)) return;
    constexpr int BS = PR_SMALL_BLOCK, WPB = BS / WAVE;
    const BinSizes c = bin_sizes(dcount, c0, c1, 0);
    const int nb1 = (c.c1 + WPB - 1) / WPB, nb0 = (c.c0 + BS - 1) / BS;
    const int total = nb1 + nb0;
    unsigned long long bytes = 0;  // thread items per thread, wave items on lane 0
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {  // block-uniform roles
        if (vb < nb1) {
            const int w = vb * WPB + (int)threadIdx.x / WAVE;
            if (w < c.c1) {  // whole waves
                bytes += pr_wave_item<PULL>(g, bcast(wl1[w]), kc);
            }
        } else {
            const int i = (vb - nb1) * BS + (int)threadIdx.x;
            if (i < c.c0) bytes += pr_thread_item<PULL>(g, wl0[i], kc);
        }
    }
    if (g.count_bytes) {
        const unsigned long long b = wave_sum_u64(bytes);
        if (lane_id() == 0 && b) add_bytes(g, KC_PR, b);
    }
}

// ---- remove invalid edges (Algorithm 3) ------------------------------------
//
// Every residual slot u->v with h(u) > h(v) + 1 is saturated: its whole
// residual moves to v regardless of e(u), so e(u) may turn negative.

// Slots sub, sub + GROUP, ... of u's row; returns the amount that left u
// (the caller subtracts it from e(u)) and adds its bytes to *bytes.  RIE_UNROLL
// slot loads per lane are issued before their height gathers.
constexpr int RIE_UNROLL = 4;

template <int GROUP>
__device__ __forceinline__ long long rie_item(DevGraph& g, int u, int sub, unsigned long long* bytes) {
    int beg = g.row_ptr[u];
    int end = beg + g.row_len[u];
    int hu = g.h[u];
    long long moved = 0;
    for (int j0 = beg + sub; j0 < end; j0 += GROUP * RIE_UNROLL) {
        unsigned long long sv[RIE_UNROLL];
#pragma unroll
        for (int q = 0; q < RIE_UNROLL; ++q) {
            int j = j0 + q * GROUP;
            sv[q] = j < end ? ld_slot(g.cr, j) : 0ull;
        }
        int hv[RIE_UNROLL];
#pragma unroll
        for (int q = 0; q < RIE_UNROLL; ++q)
            hv[q] = (int32_t)(sv[q] >> 32) > 0 ? g.h[(int)(unsigned)sv[q]] : INT_MAX;
#pragma unroll
        for (int q = 0; q < RIE_UNROLL; ++q) {
            if (hv[q] == INT_MAX || hu <= hv[q] + 1) continue;
            int j = j0 + q * GROUP;
            int32_t x = xchg_res(g.cr, j, 0);
            if (x > 0) {
                add_res(g.cr, g.rev[j], x);
                gain_e(g, (int)(unsigned)sv[q], x);
                moved += x;
                *bytes += 32;
            }
        }
    }
    if (sub == 0) *bytes += 16 + 12ull * (unsigned long long)(end - beg);
    return moved;
}


// Remove-invalid-edges for a round's three bins in one launch (256-thread
// workgroups taking virtual blocks as in k_pr_small, the workgroup bin's
// rows first, one per block).
__global__ void __launch_bounds__(256) k_rie_round(DevGraph g, const int32_t* wl0, const int32_t* wl1,
                                                   const int32_t* wl2, int c0, int c1, int c2,
                                                   DevCounters* ctr, const int32_t* dcount) {
    (void)ctr;
    constexpr int BS = 256, WPB = BS / WAVE;
    if (halted(g)) return;
    const BinSizes c = bin_sizes(dcount, c0, c1, c2);
    const int nb2 = c.c2, nb1 = (c.c1 + WPB - 1) / WPB, nb0 = (c.c0 + BS - 1) / BS;
    const int total = nb2 + nb1 + nb0;
    unsigned long long bytes = 0;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {  // block-uniform roles
        if (vb < nb2) {
            const int u = wl2[vb];
            if (g.relab && !bit_of(g.relab, u)) continue;  // block-uniform: h(u) kept, no invalid out-slot
            const long long moved = wave_sum_i64(rie_item<BS>(g, u, (int)threadIdx.x, &bytes));
            if (lane_id() == 0 && moved) add_e(g.e, u, -moved);
        } else if (vb < nb2 + nb1) {
            const int item = (vb - nb2) * WPB + (int)threadIdx.x / WAVE;
            if (item < c.c1) {  // whole waves
                const int u = wl1[item];
                if (!g.relab || bit_of(g.relab, u)) {
                    const long long moved = wave_sum_i64(rie_item<WAVE>(g, u, lane_id(), &bytes));
                    if (lane_id() == 0 && moved) add_e(g.e, u, -moved);
                }
            }
        } else {
            const int i = (vb - nb2 - nb1) * BS + (int)threadIdx.x;
            if (i < c.c0) {
                const int u = wl0[i];
                if (!g.relab || bit_of(g.relab, u)) {
                    const long long moved = rie_item<1>(g, u, 0, &bytes);
                    if (moved) add_e(g.e, u, -moved);
                }
            }
        }
    }
    if (g.count_bytes) {
        const unsigned long long b = wave_sum_u64(bytes);
        if (lane_id() == 0 && b) add_bytes(g, KC_RIE, b);
    }
}

// ---- batch of updates (Algorithm 5, first loops) ---------------------------

__device__ __forceinline__ unsigned long long pair_hash(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Locate the slot of update i = (u,v): binary search over the sorted part
// of row u, then a scan of its inserted tail.  Present: slot_of = j and the
// update index competes for win[j] (largest index = last update wins).
// Absent: the unordered pair goes into a hash table; the first thread to
// claim an entry reserves one slack slot in each of the two rows.
__device__ __forceinline__ void batch_locate_one(const DevGraph& g, const mf_update* upd, int i,
                                                 int32_t* slot_of, int32_t* win, const BatchTable& tb,
                                                 int32_t* need, DevCounters* ctr) {
    mf_update up = upd[i];
    const int N = g.n;
    if (up.u < 0 || up.u >= N || up.v < 0 || up.v >= N || up.u == up.v || up.cap < 0) {
        atomicOr(&ctr->err, 1);
        slot_of[i] = INT_MIN;
        return;
    }
    int beg = g.row_ptr[up.u];
    int lo = 0, hi = g.row_sorted[up.u];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (g.cr[beg + mid].x < up.v) lo = mid + 1;
        else hi = mid;
    }
    int j = -1;
    if (lo < g.row_sorted[up.u] && g.cr[beg + lo].x == up.v) {
        j = beg + lo;
    } else {
        int len = g.row_len[up.u];
        for (int q = g.row_sorted[up.u]; q < len; ++q)
            if (g.cr[beg + q].x == up.v) { j = beg + q; break; }
    }
    if (j >= 0) {
        slot_of[i] = j;
        atomicMax(&win[j], i);
        return;
    }
    int a = min(up.u, up.v), b = max(up.u, up.v);
    unsigned long long key = ((unsigned long long)(unsigned)a << 32) | (unsigned)b;
    unsigned mask = (unsigned)tb.capacity - 1u;
    unsigned idx = (unsigned)pair_hash(key) & mask;
    for (;;) {
        unsigned long long old = atomicCAS(&tb.key[idx], EMPTY_KEY, key);
        if (old == EMPTY_KEY) {
            int pa = atomicAdd(&need[a], 1);
            int pb = atomicAdd(&need[b], 1);
            int sa = g.row_ptr[a] + g.row_len[a] + pa;
            int sb = g.row_ptr[b] + g.row_len[b] + pb;
            if (sa >= g.row_ptr[a + 1] || sb >= g.row_ptr[b + 1]) atomicOr(&ctr->overflow, 1);
            tb.slot[2 * idx] = sa;
            tb.slot[2 * idx + 1] = sb;
            atomicAdd(&ctr->new_pairs, 1);
            break;
        }
        if (old == key) break;
        idx = (idx + 1) & mask;
    }
    slot_of[i] = -(int)(idx + 1);
    atomicMax(&tb.win[2 * idx + (up.u == a ? 0 : 1)], i);
}

__device__ __forceinline__ int winning_cap(const mf_update* upd, int32_t w, int32_t current) {
    return w >= 0 ? upd[w].cap : current;
}

// Capacity-range check of every pair a winner touches: c(u,v) + c(v,u) must
// stay within int32 (residuals of the pair sum to it).
__device__ __forceinline__ void batch_check_one(const DevGraph& g, const mf_update* upd, int i,
                                                const int32_t* slot_of, const int32_t* win,
                                                const BatchTable& tb, DevCounters* ctr) {
    int sl = slot_of[i];
    if (sl == INT_MIN) return;
    long long c1, c2;
    if (sl >= 0) {
        if (win[sl] != i) return;
        int r = g.rev[sl];
        c1 = upd[i].cap;
        c2 = winning_cap(upd, win[r], g.cap[r]);
    } else {
        int idx = -sl - 1;
        c1 = winning_cap(upd, tb.win[2 * idx], 0);
        c2 = winning_cap(upd, tb.win[2 * idx + 1], 0);
    }
    if (c1 + c2 > (long long)INT_MAX) atomicOr(&ctr->cap_overflow, 1);
}

// Write both slots of new pair `idx` (capacity 0, residual 0, paired by rev)
// and extend the two rows.
__device__ __forceinline__ void batch_insert_one(const DevGraph& g, const BatchTable& tb, int idx) {
    unsigned long long key = tb.key[idx];
    if (key == EMPTY_KEY) return;
    int a = (int)(key >> 32), b = (int)(key & 0xFFFFFFFFu);
    int sa = tb.slot[2 * idx], sb = tb.slot[2 * idx + 1];
    g.cr[sa] = make_int2(b, 0);
    g.cap[sa] = 0;
    g.capsum[sa] = 0;
    g.rev[sa] = sb;
    g.cr[sb] = make_int2(a, 0);
    g.cap[sb] = 0;
    g.capsum[sb] = 0;
    g.rev[sb] = sa;
    atomicAdd(&g.row_len[a], 1);
    atomicAdd(&g.row_len[b], 1);
}

// c_f(u,v) += c' - c (Algorithm 5, first loop), by the winning update only.
__device__ __forceinline__ void batch_apply_one(const DevGraph& g, const mf_update* upd, int i,
                                                const int32_t* slot_of, const int32_t* win,
                                                const BatchTable& tb, int32_t* touched) {
    int sl = slot_of[i];
    int j = -1;
    if (sl >= 0) {
        if (win[sl] == i) j = sl;
    } else {
        int idx = -sl - 1;
        int dir = upd[i].u < upd[i].v ? 0 : 1;
        if (tb.win[2 * idx + dir] == i) j = tb.slot[2 * idx + dir];
    }
    touched[i] = j;
    if (j < 0) return;
    int32_t c = upd[i].cap;
    int32_t delta = c - g.cap[j];
    g.cap[j] = c;
    if (delta) {
        add_res(g.cr, j, delta);
        atomicAdd(&g.capsum[j], delta);
        atomicAdd(&g.capsum[g.rev[j]], delta);
    }
}

// Over-capacity flow goes back (Algorithm 5, second loop): if c_f(u,v) < 0,
// c_f(v,u) += c_f(u,v) and c_f(u,v) = 0; the excess of u rises and that of v
// falls by the same amount (the excess recomputation of Algorithm 5, kept
// incrementally).  Of a pair's two slots at most one can be negative, since
// their residuals sum to c(u,v) + c(v,u) >= 0.
__device__ __forceinline__ void batch_clamp_one(const DevGraph& g, const mf_update* upd, int i,
                                                const int32_t* touched) {
    int j = touched[i];
    if (j < 0) return;
    int32_t r = ld_res(g.cr, j);
    if (r < 0) {
        int32_t x = -r;
        add_res(g.cr, j, x);
        add_res(g.cr, g.rev[j], -x);
        add_e(g.e, upd[i].u, x);
        add_e(g.e, upd[i].v, -x);
    }
}

// Scratch back to its idle state: win[] = -1, table empty, need[] = 0.
__device__ __forceinline__ void batch_cleanup_one(const BatchTable& tb, int32_t* need,
                                                  const int32_t* slot_of, int32_t* win, int64_t i,
                                                  int64_t k) {
    if (i < k) {
        int sl = slot_of[i];
        if (sl >= 0) win[sl] = -1;
    }
    if (i < tb.capacity) {
        unsigned long long key = tb.key[i];
        if (key != EMPTY_KEY) {
            need[(int)(key >> 32)] = 0;
            need[(int)(key & 0xFFFFFFFFu)] = 0;
            tb.key[i] = EMPTY_KEY;
        }
        tb.win[2 * i] = -1;
        tb.win[2 * i + 1] = -1;
    }
}

__global__ void __launch_bounds__(256) k_batch_locate(DevGraph g, const mf_update* upd, int64_t k,
                                                      int32_t* slot_of, int32_t* win, BatchTable tb,
                                                      int32_t* need, DevCounters* ctr) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) batch_locate_one(g, upd, (int)i, slot_of, win, tb, need, ctr);
}

__global__ void __launch_bounds__(256) k_batch_check(DevGraph g, const mf_update* upd, int64_t k,
                                                     const int32_t* slot_of, const int32_t* win,
                                                     BatchTable tb, DevCounters* ctr) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) batch_check_one(g, upd, (int)i, slot_of, win, tb, ctr);
}

// The kernels queued behind the batch's validation without the host reading
// its outcome first: each leaves at once when the validation rejected the
// batch (an invalid update, a capacity sum beyond int32, a row without room
// for its inserts), so a rejected batch changes nothing.
__device__ __forceinline__ bool batch_rejected(const DevCounters* ctr) {
    return (ctr->err | ctr->cap_overflow | ctr->overflow) != 0;
}

__global__ void __launch_bounds__(256) k_batch_insert(DevGraph g, BatchTable tb, const DevCounters* ctr,
                                                      long long* nslots) {
    if (batch_rejected(ctr)) return;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < tb.capacity) batch_insert_one(g, tb, idx);
    // the used slot count the loop kernels read: two per inserted pair
    if (idx == 0 && nslots && ctr->new_pairs)
        atomicAdd(reinterpret_cast<unsigned long long*>(nslots), 2ull * (unsigned long long)ctr->new_pairs);
}

__global__ void __launch_bounds__(256) k_batch_apply(DevGraph g, const mf_update* upd, int64_t k,
                                                     const int32_t* slot_of, const int32_t* win,
                                                     BatchTable tb, int32_t* touched, const DevCounters* ctr) {
    if (batch_rejected(ctr)) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) batch_apply_one(g, upd, (int)i, slot_of, win, tb, touched);
}

__global__ void __launch_bounds__(256) k_batch_clamp(DevGraph g, const mf_update* upd, int64_t k,
                                                     const int32_t* touched, const DevCounters* ctr) {
    if (batch_rejected(ctr)) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) batch_clamp_one(g, upd, (int)i, touched);
}

// ctr not null: leaves the scratch as it is when a row ran out of room (the
// re-layout reads the rows' demand in need[]; the host cleans up after it).
__global__ void __launch_bounds__(256) k_batch_cleanup(BatchTable tb, int32_t* need,
                                                       const int32_t* slot_of, int32_t* win,
                                                       int64_t k, const DevCounters* ctr) {
    if (ctr && ctr->overflow) return;
    batch_cleanup_one(tb, need, slot_of, win, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, k);
}

// ---- batched solve: one block per graph ---------------------------------------
// (256, 512 or 1024 threads per graph, a tuning choice)

// The whole loop of Algorithms 1 and 5 for one graph inside one block: the
// same level, worklist, push-relabel and remove-invalid-edges bodies as the
// single-graph kernels, with block barriers where those have launch
// boundaries (a workgroup barrier orders this block's global memory).
template <int BS>
__device__ void solve_graph(GraphSlot& S, int mode, const GrTune& tune) {
    __shared__ int s_cnt[4];
    __shared__ long long s_val;
    const Par P{0, 1};
    DevGraph g = S.g;
    DevCounters* ctr = S.ctr;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int N = g.n;
    if (mode == 0) {
        // Algorithm 1's initialisation: zero flow, then saturate s
        int sb = g.row_ptr[0], se = g.row_ptr[N];
        for (int j = sb + tid; j < se; j += BS) g.cr[j].y = g.cap[j];
        for (int v = tid; v < N; v += BS) {
            g.e[v] = 0;
            g.h[v] = 0;
        }
        __syncthreads();
    }
    if (mode == 0 || mode == 1) {
        int beg = g.row_ptr[g.s], len = g.row_len[g.s];
        long long sent = 0;
        for (int q = tid; q < len; q += BS) {
            int j = beg + q;
            int32_t x = g.cr[j].y;
            if (x > 0) {
                g.cr[j].y = 0;
                add_res(g.cr, g.rev[j], x);
                add_e(g.e, g.cr[j].x, x);
                sent += x;
            }
        }
        long long tot = block_sum_i64<BS>(sent);
        if (tid == 0 && tot) add_e(g.e, g.s, -tot);
        __syncthreads();
    }
    bool sweep = mode == 1 && S.warm;  // one push-relabel sweep on the previous heights
    int iters = 0;
    int status = 0;
    int rounds_left = 0;               // push-relabel rounds still due before the next relabel
    for (;;) {
        const bool relabel = !sweep && rounds_left == 0;
        int depth = 0;
        if (relabel) {
            // global relabel (Algorithm 6), then the worklist and value
            if (tid < 3) {
                ctr->front[tid] = 0;
                ctr->unv[tid] = 0;
            }
            if (tid < 4) ctr->wl[tid] = 0;
            if (tid == 0) {
                ctr->deficit_sum = 0;
                ctr->e_t = 0;
            }
            for (int i = tid; i < 4 * S.bits.nwords; i += BS) S.bits.visited[i] = 0u;
            __syncthreads();
            gr_init_body(P, g, S.q0, ctr, S.bits, 1);
            __syncthreads();
            for (int lv = 0; lv <= N; ++lv) {
                int cnt = gr_level_step<false, BS, false>(P, g, lv, (lv & 1) ? S.q1 : S.q0, (lv & 1) ? S.q0 : S.q1,
                                                   ctr, S.bits, tune, nullptr);
                __syncthreads();
                if (cnt == 0) break;
                depth = lv + 1;
            }
        } else {
            if (tid < 4) ctr->wl[tid] = 0;
            if (tid == 0) {
                ctr->deficit_sum = 0;
                ctr->e_t = 0;
            }
            __syncthreads();
        }
        worklist_body<BS>(P, g, S.wl0, S.wl1, S.wl2, ctr, 0, 1);
        __syncthreads();
        if (tid == 0) {
            for (int b = 0; b < 4; ++b) s_cnt[b] = ctr->wl[b];
            s_val = ctr->e_t + ctr->deficit_sum;
        }
        __syncthreads();
        const int c0 = s_cnt[0], c1 = s_cnt[1], c2 = s_cnt[2], active = s_cnt[3];
        if (relabel) {
            if (active == 0) break;
            if (++iters > S.max_iter) {
                status = MF_ERR_NOT_CONVERGED;
                break;
            }
            rounds_left = depth / S.round_div > 1 ? depth / S.round_div : 1;
        } else if (!sweep && active == 0) {
            // a round after a relabel left no active vertex: its push-relabel
            // and remove-invalid-edges kept the labelling valid, so if every
            // deficient vertex is still at height 0 no vertex with excess can
            // reach t or a deficit and s_val is the value; else the next
            // relabel decides
            long long raised = 0;
            for (int v = tid; v < N; v += BS)
                raised += v != g.s && v != g.t && g.e[v] < 0 && g.h[v] != 0;
            raised = block_sum_i64<BS>(raised);
            if (tid == 0) s_cnt[0] = raised != 0;
            __syncthreads();
            const bool stop = s_cnt[0] == 0;
            __syncthreads();
            if (stop) break;
            rounds_left = 0;
            continue;
        }
        sweep = false;
        if (rounds_left > 0) --rounds_left;
        // push-relabel (Algorithm 2) over the three degree bins
        unsigned long long pb = 0;  // algorithmic bytes (counted while profiling)
        for (int i = tid; i < c0; i += BS) pb += pr_thread_item<false>(g, S.wl0[i], S.kc);
        for (int i = tid / WAVE; i < c1; i += BS / WAVE) pb += pr_wave_item<false>(g, bcast(S.wl1[i]), S.kc);
        for (int i = 0; i < c2; ++i) pb += pr_block_item<false, BS>(g, S.wl2[i], S.kc_long);
        if (g.count_bytes) {
            const unsigned long long b = wave_sum_u64(pb);
            if (lane == 0 && b) add_bytes(g, KC_PR, b);
        }
        __syncthreads();
        // remove invalid edges (Algorithm 3)
        unsigned long long nb = 0;
        for (int i = tid; i < c0; i += BS) {
            int u = S.wl0[i];
            long long moved = rie_item<1>(g, u, 0, &nb);
            if (moved) add_e(g.e, u, -moved);
        }
        for (int i = tid / WAVE; i < c1; i += BS / WAVE) {
            int u = bcast(S.wl1[i]);
            long long moved = wave_sum_i64(rie_item<WAVE>(g, u, lane, &nb));
            if (lane == 0 && moved) add_e(g.e, u, -moved);
        }
        for (int i = 0; i < c2; ++i) {
            int u = S.wl2[i];
            long long moved = wave_sum_i64(rie_item<BS>(g, u, tid, &nb));
            if (lane == 0 && moved) add_e(g.e, u, -moved);
        }
        if (g.count_bytes) {
            const unsigned long long b = wave_sum_u64(nb);
            if (lane == 0 && b) add_bytes(g, KC_RIE, b);
        }
        __syncthreads();
    }
    if (tid == 0) {
        S.value = s_val;
        S.status = status;
        S.iterations = iters;
    }
}

template <int BS>
__global__ void __launch_bounds__(BS) k_batch_solve(GraphSlot* slots, const int32_t* order, int mode,
                                                    GrTune tune) {
    solve_graph<BS>(slots[order[blockIdx.x]], mode, tune);
}

// Batched repair, step 1 (one block per graph): validate and locate the
// graph's updates, then check the capacity range of the winners.
template <int BS>
__global__ void __launch_bounds__(BS) k_batch_locate_multi(GraphSlot* slots, GraphUpdates* gu) {
    GraphSlot& S = slots[blockIdx.x];
    const GraphUpdates U = gu[blockIdx.x];
    if (threadIdx.x == 0) {
        S.ctr->err = 0;
        S.ctr->overflow = 0;
        S.ctr->new_pairs = 0;
        S.ctr->cap_overflow = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < U.k; i += BS)
        batch_locate_one(S.g, U.upd, i, U.slot_of, U.win, U.tb, U.need, S.ctr);
    __syncthreads();
    for (int i = threadIdx.x; i < U.k; i += BS)
        batch_check_one(S.g, U.upd, i, U.slot_of, U.win, U.tb, S.ctr);
}

template <int BS>
__device__ __forceinline__ void cleanup_graph(const GraphUpdates& U) {
    int64_t items = U.k > U.tb.capacity ? U.k : U.tb.capacity;
    for (int64_t i = threadIdx.x; i < items; i += BS) batch_cleanup_one(U.tb, U.need, U.slot_of, U.win, i, U.k);
}

// Batched repair, step 2 (one block per graph, largest first): the rest of
// Algorithm 5 for this graph, then its loop.
template <int BS>
__global__ void __launch_bounds__(BS) k_batch_repair_multi(GraphSlot* slots, GraphUpdates* gu,
                                                           const int32_t* order, GrTune tune) {
    const int gi = order[blockIdx.x];
    GraphSlot& S = slots[gi];
    const GraphUpdates U = gu[gi];
    for (int idx = threadIdx.x; idx < U.tb.capacity; idx += BS) batch_insert_one(S.g, U.tb, idx);
    __syncthreads();
    for (int i = threadIdx.x; i < U.k; i += BS) batch_apply_one(S.g, U.upd, i, U.slot_of, U.win, U.tb, U.touched);
    __syncthreads();
    for (int i = threadIdx.x; i < U.k; i += BS) batch_clamp_one(S.g, U.upd, i, U.touched);
    __syncthreads();
    cleanup_graph<BS>(U);
    if (threadIdx.x == 0) S.g.used_slots += 2 * (int64_t)S.ctr->new_pairs;
    __syncthreads();
    solve_graph<BS>(S, 1, tune);
}

template <int BS>
__global__ void __launch_bounds__(BS) k_batch_cleanup_multi(GraphUpdates* gu) {
    cleanup_graph<BS>(gu[blockIdx.x]);
}

// ---- cut certificate --------------------------------------------------------

__global__ void __launch_bounds__(256) k_cut(DevGraph g, uint8_t* side, unsigned long long* cut) {
    const int N = g.n;
    long long c = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gridDim.x * blockDim.x) {
        bool a = g.h[v] == N;
        side[v] = a ? 1 : 0;
        if (!a) continue;
        int beg = g.row_ptr[v], end = beg + g.row_len[v];
        for (int j = beg; j < end; ++j)
            if (g.h[g.cr[j].x] < N) c += g.cap[j];
    }
    long long tot = block_sum_i64<256>(c);
    if (threadIdx.x == 0 && tot) atomicAdd(cut, (unsigned long long)tot);
}

// ---- invariants of the residual state (diagnostics) ----------------------------
//
// Counts, over every used slot and vertex, the violations of what Section 3.1
// states for every moment between kernels: c_f >= 0; the two residuals of a
// pair sum to its two capacities; the excess of v is its net inflow,
// sum over row v of (c_f - c); the excesses sum to zero.  Also the height
// range, the residual slots that are steep (h(u) > h(v) + 1 with h(u) < |V|:
// a labelling Algorithm 3 and a fresh relabel leave valid) and the active
// vertices.  out[] as in launch_check_invariants.
__global__ void __launch_bounds__(256) k_check_invariants(DevGraph g, unsigned long long* out) {
    const int N = g.n;
    long long neg = 0, pair = 0, link = 0, exc = 0, hr = 0, steep = 0, act = 0, esum = 0;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < N; u += gridDim.x * blockDim.x) {
        const int beg = g.row_ptr[u], end = beg + g.row_len[u];
        const int hu = g.h[u];
        if (hu < 0 || hu > N) ++hr;
        long long net = 0;
        for (int j = beg; j < end; ++j) {
            const int2 cr = g.cr[j];
            const int r = g.rev[j];
            if (cr.y < 0) ++neg;
            if (r < 0 || cr.x < 0 || cr.x >= N) {
                ++link;
                continue;
            }
            if (g.rev[r] != j || g.cr[r].x != u || g.capsum[j] != g.cap[j] + g.cap[r]) ++link;
            if ((long long)cr.y + g.cr[r].y != (long long)g.capsum[j]) ++pair;
            net += (long long)cr.y - g.cap[j];
            if (cr.y > 0 && hu < N && hu > g.h[cr.x] + 1) ++steep;
        }
        const long long e = g.e[u];
        if (e != net) ++exc;
        esum += e;
        if (u != g.s && u != g.t && e > 0 && hu < N) ++act;
    }
    const long long vals[8] = {neg, pair, link, exc, esum, hr, steep, act};
    for (int i = 0; i < 8; ++i) {
        const long long tot = block_sum_i64<256>(vals[i]);
        if (threadIdx.x == 0 && tot) atomicAdd(&out[i], (unsigned long long)tot);
    }
}

// ---- flow from residuals (Section 3.1, the three cases per pair) --------------

// For a completed flow: f(u,v) = c(u,v) - c_f(u,v) when positive, else 0.
// flow_slot[j] gets that value for every used slot with c > 0 and -1 for the
// rest; *count gets the number of such slots.
__global__ void __launch_bounds__(256) k_flow_slots(DevGraph g, int32_t* flow_slot,
                                                    unsigned long long* count) {
    const int N = g.n;
    long long c = 0;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < N; u += gridDim.x * blockDim.x) {
        int beg = g.row_ptr[u], len = g.row_len[u], cap_end = g.row_ptr[u + 1];
        for (int j = beg; j < cap_end; ++j) {
            int f = -1;
            if (j < beg + len && g.cap[j] > 0) {
                int d = g.cap[j] - g.cr[j].y;
                f = d > 0 ? d : 0;
                ++c;
            }
            if (flow_slot) flow_slot[j] = f;
        }
    }
    long long tot = block_sum_i64<256>(c);
    if (threadIdx.x == 0 && tot) atomicAdd(count, (unsigned long long)tot);
}

// Sum the per-block byte partials of each class into ctr->bytes and clear them.
__global__ void __launch_bounds__(256) k_reduce_bytes(DevGraph g, DevCounters* ctr) {
    const int cls = blockIdx.x;
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < BYTES_SLOTS; i += 256) {
        s += g.bytes_part[cls * BYTES_SLOTS + i];
        g.bytes_part[cls * BYTES_SLOTS + i] = 0;
    }
    __shared__ unsigned long long part[256 / WAVE];
    s = wave_sum_u64(s);
    if (lane_id() == 0) part[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 256 / WAVE; ++w) t += part[w];
        ctr->bytes[cls] = t;
    }
}

// ---- self-test of the wave primitives ---------------------------------------

__global__ void k_selftest(int* fails) {
    int lane = lane_id();
    for (int trial = 0; trial < 64; ++trial) {
        unsigned long long x = pair_hash((unsigned long long)(trial * 131 + lane * 7 + 1));
        if (trial % 3 == 0 && lane % 5 != trial % 5) x = ~0ull;  // sparse candidates
        if (trial % 7 == 0) x = ~0ull;                          // no candidate at all
        unsigned long long got = wave_min_u64(x);
        unsigned long long want = ~0ull;
        for (int l = 0; l < WAVE; ++l) {
            unsigned long long y = __shfl(x, l, WAVE);
            if (y < want) want = y;
        }
        if (got != want) atomicAdd(fails, 1);
        int tot;
        int ex = wave_excl_scan(lane % 3 + trial % 2, &tot);
        int want_ex = 0, want_tot = 0;
        for (int l = 0; l < WAVE; ++l) {
            int v = l % 3 + trial % 2;
            if (l < lane) want_ex += v;
            want_tot += v;
        }
        if (ex != want_ex || tot != want_tot) atomicAdd(fails, 1);
    }
}

inline int grid_for(int64_t items, int block, int cap = 4096) {
    int64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ---- worklist of a round without a relabel ------------------------------------
//
// The previous worklist's vertices and the ones activated by the round's
// pushes and saturations (DevGraph::act), kept when active (e > 0, h < n),
// each once (mark[v] == epoch), binned by row length.
__global__ void __launch_bounds__(256) k_next_worklist(DevGraph g, const int32_t* in0, const int32_t* in1,
                                                       const int32_t* in2, int c0, int c1, int c2, int32_t* out0,
                                                       int32_t* out1, int32_t* out2, int32_t* mark,
                                                       const int32_t* epoch_p, DevCounters* ctr) {
    if (halted(g)) return;
    const int32_t epoch = *epoch_p;
    if (c0 < 0) {  // the input lists' sizes on the device (set aside by k_zero_counts)
        c0 = ctr->wl_in[0];
        c1 = ctr->wl_in[1];
        c2 = ctr->wl_in[2];
    }
    // more activations than the list holds: some were dropped, so every
    // vertex is examined instead (the result must be the exact active set: an
    // empty one ends the loop)
    const bool all = *g.act_cnt > g.act_cap;
    const int na = min(*g.act_cnt, g.act_cap);
    const long long total = all ? (long long)g.n : (long long)c0 + c1 + c2 + na;
    for (long long base = (long long)blockIdx.x * blockDim.x; base < total;
         base += (long long)gridDim.x * blockDim.x) {
        const long long i = base + threadIdx.x;
        int v = -1;
        if (i < total) {
            if (all) v = (int)i;
            else if (i < c0) v = in0[i];
            else if (i < (long long)c0 + c1) v = in1[i - c0];
            else if (i < (long long)c0 + c1 + c2) v = in2[i - c0 - c1];
            else v = g.act[i - c0 - c1 - c2];
        }
        bool act = false;
        int bin = 0;
        if (v >= 0 && v != g.s && v != g.t && v != g.pinned && ld_e(g.e, v) > 0 && g.h[v] < g.n &&
            atomicExch(&mark[v], epoch) != epoch) {
            act = true;
            int len = g.row_len[v];
            bin = len <= g.bin0_max ? 0 : (len <= g.bin1_max ? 1 : 2);
        }
        wave_append(act && bin == 0, v, out0, &ctr->wl[0]);
        wave_append(act && bin == 1, v, out1, &ctr->wl[1]);
        wave_append(act && bin == 2, v, out2, &ctr->wl[2]);
        unsigned long long m = __ballot(act);
        if (lane_id() == 0 && m) atomicAdd(&ctr->wl[3], (int)__popcll(m));
    }
}

// The value after a round that left no active vertex.  The labelling is
// valid after every push-relabel plus remove-invalid-edges round; if every
// sink (t and each deficient vertex) is still at height 0 -- remove-invalid-
// edges can make a vertex deficient at its own height, counted here in
// round_raised -- then a vertex at |V| cannot reach a sink, no vertex with
// excess is below |V|, and the value is e(t) plus the deficits, as after a
// relabel (Algorithm 5's sum over the sinks).
__global__ void __launch_bounds__(256) k_value_if_empty(DevGraph g, DevCounters* ctr, int guard_level) {
    if (halted(g)) return;
    if (guard_level >= 0 && (ctr->front[guard_level % 3] & 0xFFFFFFFFull) != 0) return;
    if (ctr->wl[3] != 0) return;
    const int N = g.n;
    long long deficit = 0, raised = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gridDim.x * blockDim.x) {
        const int64_t ev = g.e[v];
        if (v != g.s && v != g.t && ev < 0) {
            deficit += ev;
            raised += g.h[v] != 0;
        }
        if (v == g.t) ctr->round_e_t = ev;
    }
    const long long tot = block_sum_i64<256>(deficit);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long*)&ctr->round_deficit, (unsigned long long)tot);
    const long long nr = block_sum_i64<256>(raised);
    if (threadIdx.x == 0 && nr) atomicAdd(&ctr->round_raised, (int)nr);
}

// ---- rounds on a small worklist in one workgroup ----------------------------
//
// Deep graphs (grids) run thousands of push-relabel rounds between relabels,
// each over a few hundred active vertices: as separate launches per round
// (push-relabel, remove-invalid-edges, next worklist) with a read-back each,
// the rounds cost more in launches and host round trips than in work.  Here
// one 1024-thread workgroup runs round after round with workgroup barriers
// only: push-relabel over the list (Algorithm 2), remove-invalid-edges over
// the same rows (Algorithm 3), then the next list from this one plus the
// round's activations, each vertex once (mark == epoch), binned by row
// length.  It stops after max_rounds rounds, or before a round whose list is
// empty, longer than `limit` vertices or holds a workgroup-bin row (the
// multi-block kernels take those).  Lists alternate between set a and set b
// (input in a, counts in ctr->wl); on exit ctr->wl holds the counts of the
// list to run next, ctr->rn_set which set holds it (0 a, 1 b) and
// ctr->rn_rounds the rounds run.  Activations of the last round are already
// in that list (the caller clears the activation count).
constexpr int RN_BLOCK = 1024;

__global__ void __launch_bounds__(RN_BLOCK) k_rounds_narrow(DevGraph g, int32_t* a0, int32_t* a1, int32_t* a2,
                                                           int32_t* b0, int32_t* b1, int32_t* b2, int32_t* mark,
                                                           int32_t* epoch, DevCounters* ctr, int kc, int max_rounds,
                                                           int limit) {
    if (halted(g)) return;
    constexpr int BS = RN_BLOCK;
    __shared__ int s_c[3];
    __shared__ int s_n[3];
    __shared__ int s_ep;
    __shared__ int s_na;
    __shared__ int s_act;  // the round's activations: counted in LDS (one workgroup)
    const int tid = threadIdx.x;
    const int lane = lane_id();
    DevGraph gl = g;
    gl.act_cnt = &s_act;
    if (tid < 3) s_c[tid] = ctr->wl[tid];
    if (tid == 0) s_ep = *epoch;  // moved on here once per round, stored back at the end
    __syncthreads();
    int set = 0, r = 0;
    for (; r < max_rounds; ++r) {
        const int c0 = s_c[0], c1 = s_c[1], c2 = s_c[2];
        if (c2 != 0 || c0 + c1 == 0 || c0 + c1 > limit) break;
        const int32_t* in0 = set ? b0 : a0;
        const int32_t* in1 = set ? b1 : a1;
        int32_t* out[3] = {set ? a0 : b0, set ? a1 : b1, set ? a2 : b2};
        if (tid == 0) s_act = 0;
        __syncthreads();
        // push-relabel (Algorithm 2): one thread per short row, one wave per longer row
        for (int i = tid; i < c0; i += BS) pr_thread_item<false>(gl, in0[i], kc);
        for (int w = tid / WAVE; w < c1; w += BS / WAVE) pr_wave_item<false>(gl, bcast(in1[w]), kc);
        __syncthreads();
        // remove invalid edges (Algorithm 3) over the same rows
        unsigned long long nb = 0;
        for (int i = tid; i < c0; i += BS) {
            const int u = in0[i];
            const long long moved = rie_item<1>(gl, u, 0, &nb);
            if (moved) add_e(g.e, u, -moved);
        }
        for (int w = tid / WAVE; w < c1; w += BS / WAVE) {
            const int u = bcast(in1[w]);
            const long long moved = wave_sum_i64(rie_item<WAVE>(gl, u, lane, &nb));
            if (lane == 0 && moved) add_e(g.e, u, -moved);
        }
        // every wave's activations are counted before the count is read
        __syncthreads();
        if (tid == 0) {
            ++s_ep;
            s_na = s_act;
        }
        if (tid < 3) s_n[tid] = 0;
        __syncthreads();
        // the next list: this one and the round's activations, still active,
        // each once; every vertex when activations overflowed the list
        const int ep = s_ep;
        const bool all = s_na > g.act_cap;
        const long long total = all ? (long long)g.n : (long long)c0 + c1 + s_na;
        for (long long i = tid; i < total; i += BS) {
            int v;
            if (all) v = (int)i;
            else if (i < c0) v = in0[i];
            else if (i < (long long)c0 + c1) v = in1[i - c0];
            else v = g.act[i - c0 - c1];
            if (v != g.s && v != g.t && v != g.pinned && ld_e(g.e, v) > 0 && g.h[v] < g.n &&
                atomicExch(&mark[v], ep) != ep) {
                const int len = g.row_len[v];
                const int bin = len <= g.bin0_max ? 0 : (len <= g.bin1_max ? 1 : 2);
                out[bin][atomicAdd(&s_n[bin], 1)] = v;
            }
        }
        __syncthreads();
        if (tid < 3) s_c[tid] = s_n[tid];
        set ^= 1;
        __syncthreads();
    }
    if (tid < 3) ctr->wl[tid] = s_c[tid];
    if (tid == 0) {
        ctr->wl[3] = s_c[0] + s_c[1] + s_c[2];
        ctr->rn_set = set;
        ctr->rn_rounds = r;
        *epoch = s_ep;
    }
}

// ---- relayout: rows with room for their pending inserts ---------------------
//
// Rows keep their slots in order; each row's new size is its used length plus
// the inserts it still needs plus fresh slack (rows of graphs that do not grow
// keep their size).  Vertex gv of graph i = gid[gv] sits at row_ptr[gv + i]
// (each graph's row_ptr has n_i + 1 entries).  Rows whose inserted tail is
// unsorted and that fit RL_SORT_MAX slots are sorted by column on the way.

constexpr int RL_BLOCK = 256;
constexpr int RL_SCAN_ITEMS = 16;                      // per thread
constexpr int RL_TILE = RL_BLOCK * RL_SCAN_ITEMS;      // per block
constexpr int RL_SORT_MAX = 4096;

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_sizes(RelayoutPlan p) {
    int gv = blockIdx.x * RL_BLOCK + threadIdx.x;
    if (gv >= p.V) return;
    int i = p.gid ? p.gid[gv] : 0;
    int rp = gv + i;
    int len = p.row_len[gv];
    long long sz;
    if (!p.grow || p.grow[i]) {
        long long want = (long long)len + p.need[gv];
        long long sl = (want * p.slack_pct + 99) / 100;
        sz = want + ((sl < p.slack_min ? p.slack_min : sl) << p.slack_shift);
    } else {
        sz = (long long)p.row_ptr[rp + 1] - p.row_ptr[rp];
    }
    p.size[gv] = sz;
    if (p.row_sorted[gv] < len && len <= RL_SORT_MAX) p.sort_rows[atomicAdd(p.sort_count, 1)] = gv;
}

// exclusive scan of size[0..V) into start[0..V], start[V] = total: tile sums,
// one block over the tile sums, then each tile with its offset
__device__ __forceinline__ long long block_excl_scan_i64(long long x, long long* s_w, long long* total) {
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    long long inc = x;
    for (int d = 1; d < WAVE; d <<= 1) {
        long long y = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += y;
    }
    if (lane == WAVE - 1) s_w[w] = inc;
    __syncthreads();
    long long before = 0, all = 0;
    for (int q = 0; q < RL_BLOCK / WAVE; ++q) {
        if (q < w) before += s_w[q];
        all += s_w[q];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_tile_sums(RelayoutPlan p) {
    __shared__ long long s_w[RL_BLOCK / WAVE];
    long long base = (long long)blockIdx.x * RL_TILE;
    long long x = 0;
    for (int q = 0; q < RL_SCAN_ITEMS; ++q) {
        long long idx = base + (long long)threadIdx.x * RL_SCAN_ITEMS + q;
        if (idx < p.V) x += p.size[idx];
    }
    long long total;
    block_excl_scan_i64(x, s_w, &total);
    if (threadIdx.x == 0) p.tile[blockIdx.x] = total;
}

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_scan_tiles(RelayoutPlan p, int tiles) {
    __shared__ long long s_w[RL_BLOCK / WAVE];
    long long carry = 0;
    for (int b0 = 0; b0 < tiles; b0 += RL_BLOCK) {
        int b = b0 + threadIdx.x;
        long long x = b < tiles ? p.tile[b] : 0;
        long long total;
        long long ex = block_excl_scan_i64(x, s_w, &total);
        if (b < tiles) p.tile[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) p.start[p.V] = carry;
}

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_scan(RelayoutPlan p) {
    __shared__ long long s_w[RL_BLOCK / WAVE];
    long long base = (long long)blockIdx.x * RL_TILE + (long long)threadIdx.x * RL_SCAN_ITEMS;
    long long v[RL_SCAN_ITEMS];
    long long x = 0;
    for (int q = 0; q < RL_SCAN_ITEMS; ++q) {
        v[q] = base + q < p.V ? p.size[base + q] : 0;
        x += v[q];
    }
    long long total;
    long long run = p.tile[blockIdx.x] + block_excl_scan_i64(x, s_w, &total);
    for (int q = 0; q < RL_SCAN_ITEMS; ++q) {
        if (base + q < p.V) p.start[base + q] = run;
        run += v[q];
    }
}

// src_of[j'] = old slot that moves to new slot j', or -1 for free slack
__global__ void __launch_bounds__(RL_BLOCK) k_relayout_src(RelayoutPlan p, int32_t* src_of, long long S_new) {
    long long jn = (long long)blockIdx.x * RL_BLOCK + threadIdx.x;
    if (jn >= S_new) return;
    int lo = 0, hi = p.V;                   // last row whose start <= jn
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (p.start[mid] <= jn) lo = mid;
        else hi = mid;
    }
    int gv = lo;
    int i = p.gid ? p.gid[gv] : 0;
    long long q = jn - p.start[gv];
    src_of[jn] = q < p.row_len[gv] ? (int32_t)(p.row_ptr[gv + i] + q) : -1;
}

// sort one listed row's used slots by column (columns in a row are distinct)
__global__ void __launch_bounds__(RL_BLOCK) k_relayout_sort(RelayoutPlan p, const int2* cr_old, int32_t* src_of,
                                                           int32_t* row_sorted) {
    __shared__ unsigned long long s_key[RL_SORT_MAX];
    const int gv = p.sort_rows[blockIdx.x];
    const int len = p.row_len[gv];
    const long long b = p.start[gv];
    int P2 = 1;
    while (P2 < len) P2 <<= 1;
    for (int q = threadIdx.x; q < P2; q += RL_BLOCK) {
        if (q < len) {
            int j = src_of[b + q];
            s_key[q] = ((unsigned long long)(unsigned)cr_old[j].x << 32) | (unsigned)j;
        } else {
            s_key[q] = ~0ull;
        }
    }
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
        for (int d = k >> 1; d > 0; d >>= 1) {
            for (int q = threadIdx.x; q < P2; q += RL_BLOCK) {
                int r = q ^ d;
                if (r > q) {
                    unsigned long long a = s_key[q], c = s_key[r];
                    bool up = (q & k) == 0;
                    if ((a > c) == up) {
                        s_key[q] = c;
                        s_key[r] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < len; q += RL_BLOCK) src_of[b + q] = (int32_t)(unsigned)(s_key[q] & 0xffffffffu);
    if (threadIdx.x == 0) row_sorted[gv] = len;
}

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_gather(RelayoutPlan p, const int32_t* src_of, SlotArrays from,
                                                             SlotArrays to, int32_t* where, long long S_new) {
    long long jn = (long long)blockIdx.x * RL_BLOCK + threadIdx.x;
    if (jn >= S_new) return;
    int j = src_of[jn];
    if (j >= 0) {
        to.cr[jn] = from.cr[j];
        to.cap[jn] = from.cap[j];
        to.capsum[jn] = from.capsum[j];
        where[j] = (int32_t)jn;
    } else {
        int lo = 0, hi = p.V;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (p.start[mid] <= jn) lo = mid;
            else hi = mid;
        }
        int i = p.gid ? p.gid[lo] : 0;
        int local = lo - (p.vbase ? (int)p.vbase[i] : 0);
        to.cr[jn] = make_int2(local, 0);
        to.cap[jn] = 0;
        to.capsum[jn] = 0;
        to.rev[jn] = -1;
    }
}

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_rev(const int32_t* src_of, const int32_t* rev_old,
                                                          const int32_t* where, int32_t* rev_new, long long S_new) {
    long long jn = (long long)blockIdx.x * RL_BLOCK + threadIdx.x;
    if (jn >= S_new) return;
    int j = src_of[jn];
    if (j >= 0) rev_new[jn] = where[rev_old[j]];
}

__global__ void __launch_bounds__(RL_BLOCK) k_relayout_row_ptr(RelayoutPlan p, int32_t* row_ptr) {
    int gv = blockIdx.x * RL_BLOCK + threadIdx.x;
    if (gv >= p.V) return;
    int i = p.gid ? p.gid[gv] : 0;
    row_ptr[gv + i] = (int32_t)p.start[gv];
    bool last = gv + 1 == p.V || (p.gid && p.gid[gv + 1] != i);
    if (last) row_ptr[gv + i + 1] = (int32_t)p.start[gv + 1];
}

// Atomic-throughput probe: op i adds 1 at address (i * 2654435761) mod n.
// 2654435761 is prime, so for n below it the map is a permutation of
// 0..n-1: n ops hit n distinct addresses in a scattered order.
template <class T>
__global__ void __launch_bounds__(256) k_atomic_probe(T* buf, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = (int64_t)(((unsigned long long)i * 2654435761ull) % (unsigned long long)n);
        atomicAdd(&buf[a], (T)1);
    }
}

}  // namespace

// ---- launch wrappers ----------------------------------------------------------

void launch_fill_i32(int32_t* p, int32_t value, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    k_fill_i32<<<grid_for(count, 256), 256, 0, st>>>(p, value, count);
}

void launch_reset(const DevGraph& g, int64_t slot_cap, hipStream_t st) {
    k_reset<<<grid_for(slot_cap > g.n ? slot_cap : g.n, 256, 8192), 256, 0, st>>>(g, slot_cap);
}

void launch_saturate_source(const DevGraph& g, DevCounters* ctr, hipStream_t st) {
    (void)ctr;
    k_saturate_source<<<64, 256, 0, st>>>(g);
}

void launch_saturate_sink(const DevGraph& g, hipStream_t st) {
    k_saturate_sink<<<64, 256, 0, st>>>(g);
}

void launch_mark_side(const DevGraph& g, uint8_t* side, hipStream_t st) {
    k_mark_side<<<grid_for(g.n, 256), 256, 0, st>>>(g, side);
}

void launch_saturate_cut(const DevGraph& g, const uint8_t* side, int64_t slot_cap, hipStream_t st) {
    k_saturate_cut<<<grid_for(slot_cap, 256, 8192), 256, 0, st>>>(g, side, slot_cap);
}

void launch_zero_loop_counters(DevCounters* ctr, hipStream_t st) {
    k_zero_counters_front<<<1, 64, 0, st>>>(ctr);
}

void launch_gr_init(const DevGraph& g, int2* q0, DevCounters* ctr, const GrBits& bits, int seed_deficits,
                    hipStream_t st) {
    k_zero_counters_front<<<1, 64, 0, st>>>(ctr);
    // k_gr_init writes the four bitmaps whole (no clearing launch)
    k_gr_init<<<grid_for(g.n, 256, 8192), 256, 0, st>>>(g, q0, ctr, bits, seed_deficits);
}

int gr_level_lds_bytes(int nwords, int device) {
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        return 0;
    int bytes = 4 * nwords;
    // the level kernel's own LDS (entry staging, prefix sums, deferred rows) comes on top
    const int static_bytes = 4 * (4 * GRL_BLOCK_LDS + 1 + GRL_BLOCK_LDS / WAVE + 1) + 64;
    if (bytes + static_bytes > max_lds) return 0;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gr_level<false, GRL_BLOCK_LDS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gr_level<true, GRL_BLOCK_LDS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
        return 0;
    return bytes;
}

// grid: blocks of the 256-thread variant; the LDS variant runs one block per
// 4 of those (one per CU at the default grid).
void launch_gr_level(const DevGraph& g, int level, const int2* qin, int2* qout, DevCounters* ctr,
                     const GrBits& bits, const GrTune& tune, int grid, bool forward, hipStream_t st) {
    if (tune.lds) {
        size_t shm = 4 * (size_t)bits.nwords;
        int gl = std::max(1, grid / 4);
        if (forward)
            k_gr_level<true, GRL_BLOCK_LDS><<<gl, GRL_BLOCK_LDS, shm, st>>>(g, level, qin, qout, ctr, bits, tune);
        else
            k_gr_level<false, GRL_BLOCK_LDS><<<gl, GRL_BLOCK_LDS, shm, st>>>(g, level, qin, qout, ctr, bits, tune);
    } else {
        if (forward)
            k_gr_level<true, 256><<<grid, 256, 0, st>>>(g, level, qin, qout, ctr, bits, tune);
        else
            k_gr_level<false, 256><<<grid, 256, 0, st>>>(g, level, qin, qout, ctr, bits, tune);
    }
}

void launch_gr_narrow(const DevGraph& g, int lv0, int2* q0, int2* q1, DevCounters* ctr, const GrBits& bits,
                      long long max_slots, bool forward, hipStream_t st) {
    if (forward) k_gr_narrow<true><<<1, NARROW_BLOCK, 0, st>>>(g, lv0, q0, q1, ctr, bits, max_slots);
    else k_gr_narrow<false><<<1, NARROW_BLOCK, 0, st>>>(g, lv0, q0, q1, ctr, bits, max_slots);
}

void launch_frontier_bitmap(const int2* q, int cnt, const GrBits& bits, int level, hipStream_t st) {
    launch_fill_i32(reinterpret_cast<int32_t*>(bits.fb), 0, 3 * (int64_t)bits.nwords, st);
    if (cnt > 0)
        k_mark_frontier<<<grid_for(cnt, 256), 256, 0, st>>>(q, cnt, bits.fb + (size_t)(level % 3) * bits.nwords);
}

int persistent_gr_grid(int device) {
    int coop = 0, cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gr_persistent<false>, GRP_BLOCK, 0) !=
            hipSuccess || per_cu < 1)
        return 0;
    int per_cu_f = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_f, k_gr_persistent<true>, GRP_BLOCK, 0) !=
            hipSuccess || per_cu_f < 1)
        return 0;
    // one block per CU keeps the barrier's arrivals few
    (void)per_cu;
    (void)per_cu_f;
    return cus;
}

hipError_t launch_gr_persistent(const DevGraph& g, int2* q0, int2* q1, DevCounters* ctr,
                                const GrBits& bits, const GrTune& tune, int seed_deficits, bool forward,
                                int32_t* wl0, int32_t* wl1, int32_t* wl2, bool topology, int sign,
                                int grid, hipStream_t st) {
    k_zero_counters_front<<<1, 64, 0, st>>>(ctr);
    launch_fill_i32(reinterpret_cast<int32_t*>(bits.visited), 0, 4 * (int64_t)bits.nwords, st);
    DevGraph gg = g;
    GrBits bb = bits;
    GrTune tt = tune;
    int topo = topology ? 1 : 0;
    void* args[] = {&gg, &q0, &q1, &ctr, &bb, &tt, &seed_deficits, &wl0, &wl1, &wl2, &topo, &sign};
    const void* fn = forward ? reinterpret_cast<const void*>(&k_gr_persistent<true>)
                             : reinterpret_cast<const void*>(&k_gr_persistent<false>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(GRP_BLOCK), args, 0, st);
}

hipError_t launch_gr_medium(const DevGraph& g, int lv0, int2* q0, int2* q1, DevCounters* ctr, const GrBits& bits,
                            const GrTune& tune, long long max_slots, bool forward, int grid, const MedQueue& mq,
                            hipStream_t st) {
    if (!mq.q || grid < 1 || grid > MED_MAX_BLOCKS || max_slots > mq.seg) return hipErrorInvalidValue;
    DevGraph gg = g;
    GrBits bb = bits;
    GrTune tt = tune;
    tt.lds = 0;
    MedQueue mm = mq;
    launch_fill_i32(reinterpret_cast<int32_t*>(mq.rec), 0, 6 * (int64_t)grid, st);  // no record of this launch yet
    void* args[] = {&gg, &lv0, &q0, &q1, &ctr, &bb, &tt, &max_slots, &mm};
    const void* fn = forward ? reinterpret_cast<const void*>(&k_gr_medium<true>)
                             : reinterpret_cast<const void*>(&k_gr_medium<false>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(GRM_BLOCK), args, 0, st);
}

void launch_build_worklist(const DevGraph& g, int32_t* wl0, int32_t* wl1, int32_t* wl2,
                           DevCounters* ctr, bool topology, int sign, hipStream_t st, int guard_level) {
    k_build_worklist<<<grid_for(g.n, 256, 8192), 256, 0, st>>>(g, wl0, wl1, wl2, ctr, topology ? 1 : 0,
                                                              sign, guard_level);
}

constexpr int PR_SMALL_GRID = 4096;   // 256-thread workgroups: 16 per CU
constexpr int PR_BLOCK_GRID = 1024;   // 1024-thread workgroups
constexpr int RIE_ROUND_GRID = 2048;  // 256-thread workgroups

void launch_push_relabel_round(const DevGraph& g, const int32_t* const wl[3], const int cnt[3], int kc, int kc_long,
                     bool pull, hipStream_t st, const int32_t* dcount) {
    // the workgroup bin first: its rows are the longest
    if (cnt[2] > 0) {
        const int grid = dcount ? std::min(cnt[2], PR_BLOCK_GRID) : cnt[2];
        const int32_t* d2 = dcount ? dcount + 2 : nullptr;
        if (pull) k_pr_block<true><<<grid, BLOCK_PR, 0, st>>>(g, wl[2], cnt[2], kc_long, nullptr, d2);
        else k_pr_block<false><<<grid, BLOCK_PR, 0, st>>>(g, wl[2], cnt[2], kc_long, nullptr, d2);
    }
    const int64_t total = (int64_t)(cnt[1] + PR_SMALL_BLOCK / WAVE - 1) / (PR_SMALL_BLOCK / WAVE) +
                          (cnt[0] + PR_SMALL_BLOCK - 1) / PR_SMALL_BLOCK;
    if (total <= 0) return;
    const int grid = (int)std::min<int64_t>(total, dcount ? PR_SMALL_GRID : 1 << 30);
    if (pull) k_pr_small<true><<<grid, PR_SMALL_BLOCK, 0, st>>>(g, wl[0], wl[1], cnt[0], cnt[1], kc, dcount);
    else k_pr_small<false><<<grid, PR_SMALL_BLOCK, 0, st>>>(g, wl[0], wl[1], cnt[0], cnt[1], kc, dcount);
}

void launch_remove_invalid_round(const DevGraph& g, const int32_t* const wl[3], const int cnt[3], DevCounters* ctr,
                      hipStream_t st, const int32_t* dcount) {
    const int64_t total = (int64_t)cnt[2] + (cnt[1] + 3) / 4 + (cnt[0] + 255) / 256;
    if (total <= 0) return;
    const int grid = (int)std::min<int64_t>(total, dcount ? RIE_ROUND_GRID : 1 << 30);
    k_rie_round<<<grid, 256, 0, st>>>(g, wl[0], wl[1], wl[2], cnt[0], cnt[1], cnt[2], ctr, dcount);
}

void launch_clear_counters(DevCounters* ctr, hipStream_t st) {
    // counters are plain int words; a fill kernel keeps this capture-safe
    launch_fill_i32(reinterpret_cast<int32_t*>(ctr), 0, (int64_t)(sizeof(DevCounters) / 4), st);
}

void launch_batch_locate(const DevGraph& g, const mf_update* upd, int64_t k, int32_t* slot_of,
                         int32_t* win, BatchTable tb, int32_t* need, DevCounters* ctr,
                         hipStream_t st) {
    if (k <= 0) return;
    int grid = (int)((k + 255) / 256);
    k_batch_locate<<<grid, 256, 0, st>>>(g, upd, k, slot_of, win, tb, need, ctr);
    k_batch_check<<<grid, 256, 0, st>>>(g, upd, k, slot_of, win, tb, ctr);
}

void launch_batch_insert(const DevGraph& g, BatchTable tb, const DevCounters* ctr, long long* nslots,
                         hipStream_t st) {
    if (tb.capacity <= 0) return;  // no table: no batch, no pairs to insert
    k_batch_insert<<<(tb.capacity + 255) / 256, 256, 0, st>>>(g, tb, ctr, nslots);
}

void launch_batch_apply(const DevGraph& g, const mf_update* upd, int64_t k,
                        const int32_t* slot_of, int32_t* win, BatchTable tb, int32_t* touched,
                        const DevCounters* ctr, hipStream_t st) {
    if (k <= 0) return;
    k_batch_apply<<<(int)((k + 255) / 256), 256, 0, st>>>(g, upd, k, slot_of, win, tb, touched, ctr);
}

void launch_batch_clamp(const DevGraph& g, const mf_update* upd, int64_t k,
                        const int32_t* touched, const DevCounters* ctr, hipStream_t st) {
    if (k <= 0) return;
    k_batch_clamp<<<(int)((k + 255) / 256), 256, 0, st>>>(g, upd, k, touched, ctr);
}

void launch_batch_cleanup(BatchTable tb, int32_t* need, const int32_t* slot_of, int32_t* win,
                          int64_t k, const DevCounters* ctr, hipStream_t st) {
    int64_t items = k > tb.capacity ? k : tb.capacity;
    if (items <= 0) return;
    k_batch_cleanup<<<(int)((items + 255) / 256), 256, 0, st>>>(tb, need, slot_of, win, k, ctr);
}

void launch_flow_slots(const DevGraph& g, int32_t* flow_slot, unsigned long long* count,
                       hipStream_t st) {
    k_flow_slots<<<grid_for(g.n, 256, 4096), 256, 0, st>>>(g, flow_slot, count);
}

void launch_reduce_bytes(const DevGraph& g, DevCounters* ctr, hipStream_t st) {
    k_reduce_bytes<<<KC_NCLASS, 256, 0, st>>>(g, ctr);
}

void launch_check_invariants(const DevGraph& g, unsigned long long* out, hipStream_t st) {
    launch_fill_i32(reinterpret_cast<int32_t*>(out), 0, 16, st);
    k_check_invariants<<<grid_for(g.n, 256, 4096), 256, 0, st>>>(g, out);
}

void launch_cut(const DevGraph& g, uint8_t* side, unsigned long long* cut, hipStream_t st) {
    k_cut<<<grid_for(g.n, 256, 4096), 256, 0, st>>>(g, side, cut);
}

void launch_batch_solve(GraphSlot* slots, const int32_t* order, int num, int mode, const GrTune& tune,
                        int block, hipStream_t st) {
    if (num <= 0) return;
    if (block == 256) k_batch_solve<256><<<num, 256, 0, st>>>(slots, order, mode, tune);
    else if (block == 1024) k_batch_solve<1024><<<num, 1024, 0, st>>>(slots, order, mode, tune);
    else k_batch_solve<512><<<num, 512, 0, st>>>(slots, order, mode, tune);
}

void launch_batch_locate_multi(GraphSlot* slots, GraphUpdates* gu, int num, hipStream_t st) {
    if (num > 0) k_batch_locate_multi<256><<<num, 256, 0, st>>>(slots, gu);
}

void launch_batch_repair_multi(GraphSlot* slots, GraphUpdates* gu, const int32_t* order, int num,
                               const GrTune& tune, int block, hipStream_t st) {
    if (num <= 0) return;
    if (block == 256) k_batch_repair_multi<256><<<num, 256, 0, st>>>(slots, gu, order, tune);
    else if (block == 1024) k_batch_repair_multi<1024><<<num, 1024, 0, st>>>(slots, gu, order, tune);
    else k_batch_repair_multi<512><<<num, 512, 0, st>>>(slots, gu, order, tune);
}

void launch_batch_cleanup_multi(GraphUpdates* gu, int num, hipStream_t st) {
    if (num > 0) k_batch_cleanup_multi<256><<<num, 256, 0, st>>>(gu);
}

void launch_next_worklist(const DevGraph& g, const int32_t* const in[3], const int cnt[3], int32_t* out0,
                          int32_t* out1, int32_t* out2, int32_t* mark, int32_t* epoch, DevCounters* ctr,
                          hipStream_t st) {
    // cnt null: the input sizes are the worklist counts, which k_zero_counts
    // sets aside in wl_in before it clears them; it also moves the epoch on
    k_zero_counts<<<1, 64, 0, st>>>(ctr, 1, 0, epoch);
    const int64_t most = cnt ? (int64_t)cnt[0] + cnt[1] + cnt[2] + g.act_cap : (int64_t)g.n + g.act_cap;
    k_next_worklist<<<grid_for(most, 256, 2048), 256, 0, st>>>(g, in[0], in[1], in[2], cnt ? cnt[0] : -1,
                                                              cnt ? cnt[1] : 0, cnt ? cnt[2] : 0, out0, out1,
                                                              out2, mark, epoch, ctr);
}

void launch_value_if_empty(const DevGraph& g, DevCounters* ctr, int guard_level, hipStream_t st) {
    k_value_if_empty<<<grid_for(g.n, 256, 2048), 256, 0, st>>>(g, ctr, guard_level);
}

void launch_round_terms_clear(DevCounters* ctr, hipStream_t st) {
    k_zero_counts<<<1, 64, 0, st>>>(ctr, 1, 0, nullptr);
}

void launch_rounds_narrow(const DevGraph& g, int32_t* const a[3], int32_t* const b[3], int32_t* mark,
                          int32_t* epoch, DevCounters* ctr, int kc, int max_rounds, int limit, hipStream_t st) {
    k_rounds_narrow<<<1, RN_BLOCK, 0, st>>>(g, a[0], a[1], a[2], b[0], b[1], b[2], mark, epoch, ctr, kc, max_rounds,
                                           limit);
}

void launch_zero_act(DevCounters* ctr, hipStream_t st) {
    k_zero_counts<<<1, 64, 0, st>>>(ctr, 0, 1, nullptr);
}

void launch_halt_if_done(const DevCounters* ctr, int level_end, bool after_round, int32_t* halt, hipStream_t st) {
    k_halt_if_done<<<1, 64, 0, st>>>(ctr, level_end, after_round ? 1 : 0, halt);
}

void launch_set_i32(int32_t* p, int32_t value, hipStream_t st) {
    k_set_i32<<<1, 64, 0, st>>>(p, value);
}

void launch_copy_i32(int32_t* dst, const int32_t* src, int64_t count, hipStream_t st) {
    if (count > 0) k_copy_i32<<<grid_for(count, 256, 1024), 256, 0, st>>>(dst, src, count);
}

void launch_set_i64(long long* p, long long value, hipStream_t st) {
    k_set_i64<<<1, 64, 0, st>>>(p, value);
}

int64_t relayout_tiles(int32_t V) { return ((int64_t)V + RL_TILE - 1) / RL_TILE; }

void launch_relayout_plan(const RelayoutPlan& p, hipStream_t st) {
    const int tiles = (int)relayout_tiles(p.V);
    k_fill_i32<<<1, 64, 0, st>>>(p.sort_count, 0, 1);
    k_relayout_sizes<<<(p.V + RL_BLOCK - 1) / RL_BLOCK, RL_BLOCK, 0, st>>>(p);
    k_relayout_tile_sums<<<tiles, RL_BLOCK, 0, st>>>(p);
    k_relayout_scan_tiles<<<1, RL_BLOCK, 0, st>>>(p, tiles);
    k_relayout_scan<<<tiles, RL_BLOCK, 0, st>>>(p);
}

void launch_relayout_move(const RelayoutPlan& p, int32_t sort_count, int64_t S_new, SlotArrays from, SlotArrays to,
                          int32_t* src_of, int32_t* where, int32_t* row_ptr, int32_t* row_sorted, hipStream_t st) {
    const unsigned blocks = (unsigned)((S_new + RL_BLOCK - 1) / RL_BLOCK);
    k_relayout_src<<<blocks, RL_BLOCK, 0, st>>>(p, src_of, S_new);
    if (sort_count > 0) k_relayout_sort<<<sort_count, RL_BLOCK, 0, st>>>(p, from.cr, src_of, row_sorted);
    k_relayout_gather<<<blocks, RL_BLOCK, 0, st>>>(p, src_of, from, to, where, S_new);
    k_relayout_rev<<<blocks, RL_BLOCK, 0, st>>>(src_of, from.rev, where, to.rev, S_new);
    k_relayout_row_ptr<<<(p.V + RL_BLOCK - 1) / RL_BLOCK, RL_BLOCK, 0, st>>>(p, row_ptr);
}

double atomic_probe(int64_t n, int width, hipStream_t st) {
    if (n >= 2654435761ll) return -1.0;
    void* buf = nullptr;
    size_t bytes = (size_t)n * (width == 8 ? 8 : 4);
    if (hipMalloc(&buf, bytes) != hipSuccess) return -1.0;
    hipEvent_t a = nullptr, b = nullptr;
    double rate = -1.0;
    if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
        hipMemsetAsync(buf, 0, bytes, st) == hipSuccess) {
        const int grid = 4096;
        for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
            (void)hipEventRecord(a, st);
            if (width == 8) k_atomic_probe<unsigned long long><<<grid, 256, 0, st>>>((unsigned long long*)buf, n);
            else k_atomic_probe<unsigned><<<grid, 256, 0, st>>>((unsigned*)buf, n);
            (void)hipEventRecord(b, st);
        }
        float ms = 0.f;
        if (hipGetLastError() == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
            hipEventElapsedTime(&ms, a, b) == hipSuccess && ms > 0.f)
            rate = (double)n / (ms * 1e-3);
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(buf);
    return rate;
}

int device_selftest(hipStream_t st) {
    int* d = nullptr;
    if (hipMalloc(&d, sizeof(int)) != hipSuccess) return -1;
    int h = 0;
    (void)hipMemcpyAsync(d, &h, sizeof(int), hipMemcpyHostToDevice, st);
    k_selftest<<<1, 64, 0, st>>>(d);
    (void)hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(d);
    return h;
}

}  // namespace mf
