// Internal declarations shared by the host driver (api.cpp, bicsr.cpp) and
// the gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mf.h"

namespace mf {

// Bi-CSR residual graph (Section 5.1).  Row v occupies slot positions
// [row_ptr[v], row_ptr[v+1]); its first row_len[v] slots are in use, the rest
// is slack for inserted pairs.  The first row_sorted[v] slots are sorted by
// column (the rows as loaded); inserted slots follow unsorted.  Slot j holds
// {col, res} (neighbour and residual capacity u->col), its capacity cap[j]
// and the index rev[j] of the slot col->u in row col.  The two residuals of
// a pair always sum to its two capacities (Section 3.1), so capsum[j] lets a
// row scan see the reverse residual without touching the reverse slot.
struct DevGraph {
    int32_t n, s, t;
    int32_t root;    // BFS root: t for the solve, s or t while completing a flow
    int32_t pinned;  // never labelled by the BFS: s for the solve
    int32_t* row_ptr;
    int32_t* row_len;
    int32_t* row_sorted;
    int2* cr;
    int32_t* rev;
    int32_t* cap;
    int32_t* capsum;  // cap[j] + cap[rev[j]]: res[rev[j]] = capsum[j] - res[j] between sweeps
    int64_t* e;
    int32_t* h;
    int64_t used_slots;                  // sum of row_len
    const long long* nslots;             // not null: the same count in device memory, which the kernels
                                         // read instead (a captured launch keeps its arguments)
    unsigned long long* bytes_part;      // KC_NCLASS x BYTES_SLOTS algorithmic-byte partial sums
    int count_bytes;                     // 1 while kernel classes are being profiled
    int bin0_max, bin1_max;              // worklist degree bins: thread up to bin0_max slots, wave up to bin1_max
    const uint8_t* side;                 // not null: a relabel only labels vertices with side[v] == side_keep
    int side_keep;
    int32_t* act;                        // not null: push-relabel / remove-invalid-edges append every vertex
    int32_t* act_cnt;                    // whose excess turns positive, counting in *act_cnt (which may
    int32_t act_cap;                     // pass act_cap: the extra ones are dropped)
    unsigned* relab;                     // not null: push-relabel sets bit u when it raises h(u); the
                                         // worklist build clears it; remove-invalid-edges skips unset rows
    const int32_t* halt;                 // not null and set: the single-graph loop kernels leave at once
                                         // (a pipelined iteration queued behind the loop's last one)
    int32_t bfs_cap;                     // 1: a relabel that starts from a valid labelling with every sink
                                         // at height 0 stops once every vertex with excess below |V| has its
                                         // height; a vertex not reached keeps max(depth + 1, its old height)
    int32_t* h_prev;                     // ... the old heights (copied by the relabel's init)
};

// Partial sums of algorithmic bytes: a kernel block adds into slot
// blockIdx % BYTES_SLOTS of its class, so counting contends on no address.
constexpr int BYTES_SLOTS = 4096;

// Device-side counters, one block of memory read back with a single copy.
struct DevCounters {
    unsigned long long front[3];  // per BFS level (ring): entries in the low 32 bits, the
                                  // frontier's slot count in the high 32 bits
    int32_t wl[4];             // worklist sizes per degree bin
    int32_t err;               // batch: invalid update seen
    int32_t overflow;          // batch: row slack exhausted
    int32_t new_pairs;         // batch: distinct absent pairs
    int32_t cap_overflow;      // batch: c(u,v)+c(v,u) would leave int32
    int32_t levels;            // global relabel: the level after the last non-empty one so far (the
                               // BFS depth once it is over; the one-workgroup levels leave the
                               // level to continue from)
    int32_t bar_err;           // persistent global relabel: barrier gave up / level bound hit
    unsigned bar_count;        // grid barrier arrivals
    unsigned bar_gen;          // grid barrier generation
    long long unv[3];          // unvisited slots at the start of level lv in unv[lv % 3]; the
                               // relabel's init leaves the total of all labellable rows in unv[2]
    long long deficit_sum;     // sum of negative excess outside {s,t}
    long long e_t;             // e(t) at the worklist build
    unsigned long long bytes[8];  // algorithmic bytes per kernel class
    int32_t act;               // vertices appended to DevGraph::act (may exceed act_cap: then some were dropped)
    int32_t act_pad;
    unsigned long long seed_front;  // the last relabel's level-0 frontier (front[] format)
    int32_t wl_in[4];          // worklist sizes as the last next-worklist build found them (its input)
    long long round_e_t;       // value terms after a round whose next worklist came out empty:
    long long round_deficit;   // e(t) and the sum of negative excess outside {s,t}
    int32_t round_raised;      // ... and the deficient vertices above height 0 (made by remove-invalid-
                               //     edges after the relabel); the loop may end there only if none
    int32_t rn_set;            // one-workgroup rounds: which list set holds the next list (0 in, 1 other)
    int32_t rn_rounds;         // ... and how many rounds they ran
    int32_t bfs_total;         // capped relabel: vertices with excess (counted by the init)
    int32_t bfs_disc[3];       // ... of them labelled at level lv, in bfs_disc[lv % 3]
    int32_t bfs_cum[3];        // ... labelled at levels <= lv, in bfs_cum[lv % 3]
    int32_t bfs_capped;        // ... > 0: it stopped before processing level bfs_capped - 1, whose
                               //     frontier keeps that height; the rest get bfs_capped or more
    int32_t bfs_raised;        // ... deficient vertices above height 0 when it began (then no cap)
    int32_t bfs_ok;            // ... it began from a valid labelling (lab_valid, taken by the init)
    int32_t lab_valid;         // the heights are a valid labelling: set by a worklist build after a
                               // finished relabel (the rounds behind it keep it so), cleared when the
                               // next relabel starts and at the start of every solve
};

// KC_GR: multi-block BFS level launches; KC_GRS: the relabel's seeding and its
// one-workgroup thin-frontier levels
enum KernelClass { KC_GR = 0, KC_PR = 1, KC_RIE = 2, KC_WL = 3, KC_BATCH = 4, KC_INIT = 5, KC_GRS = 6, KC_NCLASS = 8 };

// Default degree bins for the worklist: rows up to BIN0_MAX slots get one
// thread, up to BIN1_MAX one wave, longer rows one 1024-thread block.
constexpr int BIN0_MAX = 16;
constexpr int BIN1_MAX = 512;
constexpr int BLOCK_PR = 1024;
// Per-workgroup queue segments of the mid-size BFS levels (one cooperative
// launch of up to MED_MAX_BLOCKS workgroups): two rings of `blocks` segments
// of `seg` entries {vertex, first slot, slots, 0} (at most MED_MAX_SEG), and
// three rings of one 64-bit record per workgroup (the two level rings and
// the hand-back's piece counts), cleared before every launch.
constexpr int MED_MAX_BLOCKS = 64;
constexpr int MED_MAX_SEG = (1 << 17) - 1;
struct MedQueue {
    int4* q;
    unsigned long long* rec;
    long long seg;
};

// Global-relabel frontier entries cover at most GR_CHUNK slots of a row.
constexpr int GR_CHUNK = 256;
// Direction rule (Beamer, Asanovic, Patterson's direction-optimizing BFS:
// alpha 14; beta 64 measured best here, their paper uses 24) and the entry
// count above which a top-down level stages the visited bitmap in LDS.
constexpr int GR_BU_ALPHA = 14;
constexpr int GR_BU_BETA = 64;
constexpr int GR_STAGE_MIN = 1024;
// Bottom-up: a thread checks this many slots of its row before handing the
// rest of a long row to a wave.
constexpr int BU_THREAD_SLOTS = 32;

// Bitmaps of one global relabel: visited (nwords words), then a ring of
// three frontier bitmaps (fb + r * nwords), all zeroed before each relabel.
struct GrBits {
    unsigned* visited;
    unsigned* fb;
    int nwords;
};

// Direction and staging knobs of the BFS levels.
struct GrTune {
    int bu_alpha;   // bottom-up when frontier slots * alpha > unvisited slots ...
    int bu_beta;    // ... and frontier vertices * beta > n; alpha <= 0 disables bottom-up
    int stage_min;  // top-down levels with at least this many entries stage the visited bitmap
    int lds;        // the bitmap fits in LDS (dynamic shared memory provided at launch)
    int bu_lb;      // bottom-up levels stream the unvisited rows slot-parallel (no per-row early exit)
    int bu_wide;    // bottom-up threads keep eight slot loads in flight instead of four
};

// One graph of a batched solve: views into the pooled device arrays (slot
// indices and rev are pool-global, vertex arrays are offset to the graph)
// plus its own scratch and result.
struct GraphSlot {
    DevGraph g;
    int2* q0;
    int2* q1;
    int32_t* wl0;
    int32_t* wl1;
    int32_t* wl2;
    GrBits bits;
    DevCounters* ctr;
    int32_t kc;
    int32_t kc_long;           // cycles for rows the workgroup takes whole (at most kc)
    int32_t warm;              // repairs: one sweep on the previous heights first
    int32_t round_div;         // push-relabel rounds per relabel: BFS depth / round_div, at least 1
    int64_t max_iter;
    // results of the last launch
    long long value;
    int32_t status;            // 0 ok, MF_ERR_NOT_CONVERGED
    int32_t iterations;
};

// Batch scratch: hash table of absent pairs, keyed by the unordered pair.
struct BatchTable {
    unsigned long long* key;   // (lo << 32 | hi), ~0 = empty
    int32_t* win;              // 2 per entry: last update index per direction (lo->hi, hi->lo)
    int32_t* slot;             // 2 per entry: reserved slot in row lo, row hi
    int32_t capacity;          // power of two
};

// One graph's share of a batched repair: its updates and scratch.
struct GraphUpdates {
    const mf_update* upd;
    int32_t k;
    int32_t* slot_of;
    int32_t* touched;
    int32_t* win;              // pool-global, per slot
    int32_t* need;             // per vertex of this graph
    BatchTable tb;
};

// Slot-sized arrays of a Bi-CSR (one graph, or a pool of graphs).
struct SlotArrays {
    int2* cr;
    int32_t* rev;
    int32_t* cap;
    int32_t* capsum;
};

// Inputs of a device relayout.  Vertex gv (0..V) belongs to graph gid[gv]
// (gid null: one graph) whose first vertex is vbase[graph] (null: 0); its
// row starts at row_ptr[gv + graph] (every graph's row_ptr has n + 1
// entries).  Rows of graphs with grow[graph] == 0 keep their size (grow
// null: every row grows); a growing row gets room for need[gv] more slots
// plus fresh slack.
struct RelayoutPlan {
    int32_t V;
    const int32_t* row_ptr;
    const int32_t* row_len;
    const int32_t* row_sorted;
    const int32_t* need;
    const int32_t* gid;
    const int64_t* vbase;
    const uint8_t* grow;
    int32_t slack_min, slack_pct;
    int32_t slack_shift;       // the fresh slack is scaled by 2^slack_shift (grows with each relayout)
    // scratch
    int64_t* size;             // V
    int64_t* start;            // V + 1
    int64_t* tile;             // relayout_tiles(V)
    int32_t* sort_rows;        // V
    int32_t* sort_count;       // 1
};

// Where a handle's device buffers come from: the caller's allocator when
// mf_options sets one, else hipMalloc / hipFree.
struct DeviceAllocator {
    void* (*alloc_fn)(size_t, void*) = nullptr;
    void (*free_fn)(void*, void*) = nullptr;
    void* ctx = nullptr;
    hipError_t allocate(void** p, size_t bytes) const {
        if (!alloc_fn) return hipMalloc(p, bytes);
        *p = alloc_fn(bytes, ctx);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    void release(void* p) const {
        if (!p) return;
        if (free_fn) free_fn(p, ctx);
        else (void)hipFree(p);
    }
};

// Tuning of a handle resolved from mf_options (0 = default).
struct Tuning {
    int32_t kc_option;   // 0: round(m/n) per graph
    GrTune gr;
    int32_t round_div;
    int32_t bin0, bin1;
    int32_t batch_block;
    int32_t long_cycles;  // push/relabel cycles of the workgroup bin (capped at kc)
};
// MF_ERR_INVALID for inconsistent fields; a field left 0 takes its default
// (the library reads no environment variable).
mf_status resolve_tuning(const mf_options& o, Tuning* t);

// ---- launch wrappers (kernels.hip) ---------------------------------------
void launch_fill_i32(int32_t* p, int32_t value, int64_t count, hipStream_t st);
void launch_reset(const DevGraph& g, int64_t slot_cap, hipStream_t st);
void launch_saturate_source(const DevGraph& g, DevCounters* ctr, hipStream_t st);
// static push-pull: every residual in-slot w->t of the sink is saturated (w may turn deficient)
void launch_saturate_sink(const DevGraph& g, hipStream_t st);
// side[v] = 1 where h[v] == n (the source side of the last terminating relabel), else 0
void launch_mark_side(const DevGraph& g, uint8_t* side, hipStream_t st);
// every residual slot u->v with side[u] == 1 and side[v] == 0 is saturated
void launch_saturate_cut(const DevGraph& g, const uint8_t* side, int64_t slot_cap, hipStream_t st);
void launch_zero_loop_counters(DevCounters* ctr, hipStream_t st);
void launch_gr_init(const DevGraph& g, int2* q0, DevCounters* ctr, const GrBits& bits, int seed_deficits,
                    hipStream_t st);
int gr_level_lds_bytes(int nwords, int device);
void launch_gr_level(const DevGraph& g, int level, const int2* qin, int2* qout, DevCounters* ctr,
                     const GrBits& bits, const GrTune& tune, int grid, bool forward, hipStream_t st);
int persistent_gr_grid(int device);
hipError_t launch_gr_persistent(const DevGraph& g, int2* q0, int2* q1, DevCounters* ctr,
                                const GrBits& bits, const GrTune& tune, int seed_deficits, bool forward,
                                int32_t* wl0, int32_t* wl1, int32_t* wl2, bool topology, int sign,
                                int grid, hipStream_t st);
// guard_level >= 0: a build queued behind BFS levels up to guard_level - 1
// does nothing unless the BFS ended there
void launch_build_worklist(const DevGraph& g, int32_t* wl0, int32_t* wl1, int32_t* wl2,
                           DevCounters* ctr, bool topology, int sign, hipStream_t st, int guard_level = -1);
void launch_clear_counters(DevCounters* ctr, hipStream_t st);
void launch_reduce_bytes(const DevGraph& g, DevCounters* ctr, hipStream_t st);
void launch_batch_locate(const DevGraph& g, const mf_update* upd, int64_t k, int32_t* slot_of,
                         int32_t* win, BatchTable tb, int32_t* need, DevCounters* ctr,
                         hipStream_t st);
// insert / apply / clamp leave at once when the validation (locate) rejected
// the batch; insert adds the new slots to *nslots (when not null)
void launch_batch_insert(const DevGraph& g, BatchTable tb, const DevCounters* ctr, long long* nslots,
                         hipStream_t st);
void launch_batch_apply(const DevGraph& g, const mf_update* upd, int64_t k,
                        const int32_t* slot_of, int32_t* win, BatchTable tb, int32_t* touched,
                        const DevCounters* ctr, hipStream_t st);
void launch_batch_clamp(const DevGraph& g, const mf_update* upd, int64_t k,
                        const int32_t* touched, const DevCounters* ctr, hipStream_t st);
// ctr not null: skipped when a row ran out of room (its demand stays in need[])
void launch_batch_cleanup(BatchTable tb, int32_t* need, const int32_t* slot_of, int32_t* win,
                          int64_t k, const DevCounters* ctr, hipStream_t st);
void launch_cut(const DevGraph& g, uint8_t* side, unsigned long long* cut, hipStream_t st);
// out[8] (device): negative residuals, broken pair sums, broken pair links,
// excess mismatches, sum of excesses, heights out of range, steep residual
// slots, active vertices
void launch_check_invariants(const DevGraph& g, unsigned long long* out, hipStream_t st);
void launch_flow_slots(const DevGraph& g, int32_t* flow_slot, unsigned long long* count,
                       hipStream_t st);
int device_selftest(hipStream_t st);
// Batched solve: one block per graph, graphs taken in `order`; mode 0 solves
// from zero flow (Algorithm 1), mode 1 resumes after applied updates
// (Algorithm 5's loop).
void launch_batch_solve(GraphSlot* slots, const int32_t* order, int num, int mode, const GrTune& tune,
                        int block, hipStream_t st);
// Batched repair, first launch: validate and locate every graph's updates.
void launch_batch_locate_multi(GraphSlot* slots, GraphUpdates* gu, int num, hipStream_t st);
// Second launch: insert, apply, clamp, clean up and resume each graph.
void launch_batch_repair_multi(GraphSlot* slots, GraphUpdates* gu, const int32_t* order, int num,
                               const GrTune& tune, int block, hipStream_t st);
// After a failed validation: scratch back to idle for every graph.
void launch_batch_cleanup_multi(GraphUpdates* gu, int num, hipStream_t st);
// thin-frontier BFS levels in one workgroup; ctr->levels = the level to continue from
void launch_gr_narrow(const DevGraph& g, int lv0, int2* q0, int2* q1, DevCounters* ctr, const GrBits& bits,
                      long long max_slots, bool forward, hipStream_t st);
// BFS levels from lv0 in one cooperative launch of `grid` 1024-thread blocks
// while the frontier covers at most max_slots slots (ctr->levels: where to
// continue; ctr->bar_err set if a grid barrier gave up)
hipError_t launch_gr_medium(const DevGraph& g, int lv0, int2* q0, int2* q1, DevCounters* ctr, const GrBits& bits,
                            const GrTune& tune, long long max_slots, bool forward, int grid, const MedQueue& mq,
                            hipStream_t st);
// zero the three frontier bitmaps, then set the current level's from its queue
void launch_frontier_bitmap(const int2* q, int cnt, const GrBits& bits, int level, hipStream_t st);
int64_t relayout_tiles(int32_t V);
// n scattered atomicAdds of `width` bytes (4 or 8) on n distinct addresses; ops/s, < 0 on failure
double atomic_probe(int64_t n, int width, hipStream_t st);
// A push-relabel round in two launches (the workgroup bin with kc_long
// cycles, then the thread and wave bins with kc) and a remove-invalid-edges
// round in one.  dcount null: the bins hold cnt[0..2] rows; else their
// sizes are dcount[0..2] on the device and cnt[] upper bounds for the grid.
void launch_push_relabel_round(const DevGraph& g, const int32_t* const wl[3], const int cnt[3], int kc, int kc_long,
                     bool pull, hipStream_t st, const int32_t* dcount = nullptr);
void launch_remove_invalid_round(const DevGraph& g, const int32_t* const wl[3], const int cnt[3], DevCounters* ctr,
                      hipStream_t st, const int32_t* dcount = nullptr);
// next worklist of a push-relabel round without a relabel: the previous
// worklist's bins (counts cnt[0..2], or with cnt null the worklist counts on
// the device, set aside in wl_in first) and the activation list, filtered to
// active vertices (e > 0, h < n), deduplicated with mark[v] == *epoch (a
// device word the launch increments first), binned
void launch_next_worklist(const DevGraph& g, const int32_t* const in[3], const int cnt[3], int32_t* out0,
                          int32_t* out1, int32_t* out2, int32_t* mark, int32_t* epoch, DevCounters* ctr,
                          hipStream_t st);
void launch_set_i64(long long* p, long long value, hipStream_t st);
// dst[0..count) = src[0..count); src may be pinned host memory's device address
void launch_copy_i32(int32_t* dst, const int32_t* src, int64_t count, hipStream_t st);
void launch_set_i32(int32_t* p, int32_t value, hipStream_t st);
// sets *halt when the iteration queued behind levels 0..level_end-1 ended the loop
// (after_round: when its first round left no active vertex)
void launch_halt_if_done(const DevCounters* ctr, int level_end, bool after_round, int32_t* halt, hipStream_t st);
void launch_zero_act(DevCounters* ctr, hipStream_t st);
// Up to max_rounds push-relabel + remove-invalid-edges rounds in one
// workgroup while the worklist holds at most `limit` vertices and no
// workgroup-bin row (input lists a with counts in ctr->wl; lists alternate
// with b; ctr->wl, rn_set and rn_rounds say where it stopped).  dg.act must be
// set, dg.relab null; epoch: the device epoch word (one per round).
void launch_rounds_narrow(const DevGraph& g, int32_t* const a[3], int32_t* const b[3], int32_t* mark,
                          int32_t* epoch, DevCounters* ctr, int kc, int max_rounds, int limit, hipStream_t st);
// the round value terms to zero (as a next-worklist build leaves them)
void launch_round_terms_clear(DevCounters* ctr, hipStream_t st);
// After a next-worklist build that found no active vertex (and, guard_level
// >= 0, a BFS that ended before guard_level): the value terms of the state,
// into round_e_t and round_deficit, and the deficient vertices above height
// 0 into round_raised (all zeroed by that build).  Otherwise nothing.
void launch_value_if_empty(const DevGraph& g, DevCounters* ctr, int guard_level, hipStream_t st);
// sizes, their scan into start[] and the rows to sort; then the caller reads
// start[V] (the new slot count) and *sort_count
void launch_relayout_plan(const RelayoutPlan& p, hipStream_t st);
// moves the slots into `to` (S_new slots), rewrites row_ptr in place and
// sets row_sorted of the rows it sorted; src_of: S_new, where: old slot count
void launch_relayout_move(const RelayoutPlan& p, int32_t sort_count, int64_t S_new, SlotArrays from, SlotArrays to,
                          int32_t* src_of, int32_t* where, int32_t* row_ptr, int32_t* row_sorted, hipStream_t st);


// ---- allocation-free repair (noalloc.hip) --------------------------------
// Largest batch the allocation-free repair takes, and its hash table's size
// (a power of two of at least twice that, as the allocating path sizes it).
constexpr int64_t NOALLOC_MAX_UPDATES = MF_NOALLOC_MAX_UPDATES;
constexpr int32_t NOALLOC_TABLE = 2 * (int32_t)MF_NOALLOC_MAX_UPDATES;
static_assert((NOALLOC_TABLE & (NOALLOC_TABLE - 1)) == 0, "table size must be a power of two");
// Views into the GPU's static scratch array (device addresses).
struct NoallocScratch {
    unsigned long long* table_key;   // NOALLOC_TABLE
    int32_t* table_win;              // 2 * NOALLOC_TABLE
    int32_t* table_slot;             // 2 * NOALLOC_TABLE
    int32_t* slot_of;                // NOALLOC_MAX_UPDATES
    int32_t* touched;                // NOALLOC_MAX_UPDATES
    size_t bytes;                    // size of the whole array
};
// The scratch array of `device`, which the caller has made current: its
// address is looked up on the first call for each device and kept.
mf_status noalloc_scratch(int device, NoallocScratch* out);

// ---- host Bi-CSR builder (bicsr.cpp) -------------------------------------
struct HostBiCSR {
    int32_t n = 0;
    std::vector<int32_t> row_ptr, row_len, row_sorted, col, rev, cap;
    int64_t pairs = 0;         // merged directed pairs with a slot
    int64_t m_unique = 0;      // merged directed pairs with capacity > 0 at load
};

// Validates and builds; returns MF_OK, MF_ERR_INVALID or MF_ERR_OVERFLOW.
mf_status build_bicsr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      const int32_t* cap, int32_t s, int32_t t, int32_t slack_min,
                      int32_t slack_pct, HostBiCSR* out);

// Device relayout (relayout.cpp): runs the plan, allocates the new slot
// arrays, moves the slots and frees the old arrays; *arrays and *S_new then
// describe the new layout and row_ptr / row_sorted (device) are rewritten.
// On error nothing has changed (MF_ERR_OVERFLOW: more than INT32_MAX - 1
// slots; MF_ERR_OUT_OF_MEMORY; MF_ERR_DEVICE).
mf_status relayout_device(RelayoutPlan p, SlotArrays* arrays, int64_t S_old, int64_t* S_new, int32_t* row_ptr,
                          int32_t* row_sorted, hipStream_t st, const DeviceAllocator& mem);


}  // namespace mf
