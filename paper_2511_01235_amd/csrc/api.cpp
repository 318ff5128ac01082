// Host driver and C ABI of the dynamic max-flow library.
//
// mf_maxflow runs Algorithm 1; mf_apply_batch runs Algorithm 5; both share
// the loop {global relabel (Algorithms 4/6), worklist (Section 5.2),
// push-relabel (Algorithm 2), remove-invalid-edges (Algorithm 3)} whose only
// host/device synchronisations are the frontier-size checks of the BFS and
// one read of the worklist size and value per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <utility>
#include <thread>
#include <vector>

#include "mf.h"
#include "mf_internal.h"

using mf::DevCounters;
using mf::DevGraph;

struct mf_graph {
    int device = 0;
    mf::DeviceAllocator mem;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mf_options opt{};
    int32_t kc = 1;
    int32_t slack_min = 2, slack_pct = 12;
    int64_t max_iter = 0;
    int32_t n = 0, s = 0, t = 0;
    int64_t pairs = 0, m_unique = 0;
    int64_t slot_cap = 0;
    DevGraph dg{};
    // device buffers
    int2* q[2] = {nullptr, nullptr};
    int64_t q_cap = 0;
    int32_t* wl[3] = {nullptr, nullptr, nullptr};
    DevCounters* ctr = nullptr;
    DevCounters* ctr_h = nullptr;  // pinned
    int32_t* win = nullptr;        // per slot, -1 when idle
    int32_t* need = nullptr;       // per vertex, 0 when idle
    int32_t* slot_of = nullptr;
    int32_t* touched = nullptr;
    mf_update* upd = nullptr;
    mf_update* upd_h = nullptr;      // pinned staging of host-memory batches (k_cap entries)
    mf_update* upd_h_dev = nullptr;  // the same buffer's device-side address
    int64_t k_cap = 0;
    mf::BatchTable tb{};
    uint8_t* side = nullptr;
    unsigned long long* cut_acc = nullptr;  // 8 words: cut / flow-slot sums, invariant counts
    // state
    bool solved = false;
    bool poisoned = false;
    int64_t last_value = 0;
    // stats
    int32_t relayouts = 0;
    int64_t last_iterations = 0, last_levels = 0, last_active_sum = 0, last_new_pairs = 0, last_rounds = 0;
    int64_t last_capped = 0;         // relabels of the last call whose BFS stopped early (bfs_cap)
    double last_ms = 0;
    uint32_t prof_mask = 0;
    double kernel_ms[8] = {0};
    int64_t kernel_launches[8] = {0};
    double kernel_bytes[8] = {0};
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    int gr_grid = 1024;
    mf::GrBits bits{};
    mf::GrTune tune{mf::GR_BU_ALPHA, mf::GR_BU_BETA, mf::GR_STAGE_MIN, 0, 0, 0};
    int persistent_grid = 0;  // > 0: global relabel as one cooperative launch of this many blocks
    int first_chunk = 7;      // BFS levels launched before the first frontier check (at least)
    bool trace_gr = false;    // option trace: one level per launch, each printed to stderr
    bool narrow_seed = true;  // start relabels in one workgroup (the last one's seeds were few enough)
    int32_t last_depth = 0;   // BFS levels of the last global relabel
    bool queue_rounds = true; // option queue_rounds: worklist build and rounds queued behind the relabel
    bool pipeline = true;     // option pipeline: a relabel iteration queued ahead of the host's read
    DevCounters* snap_h[2] = {nullptr, nullptr};  // pinned: counters of the iterations in flight
    hipEvent_t snap_ev[2] = {nullptr, nullptr};
    int32_t kc_block = 1;     // push/relabel cycles of the workgroup bin (capped at kc)
    int32_t round_div = 4;    // push-relabel rounds per global relabel: BFS depth / round_div ...
    int32_t round_max = 4096; // ... at most this many
    int32_t round_min = 2;    // ... and at least this many (option round_min)
    bool incremental_rounds = true;  // rounds take their worklist from the previous one plus activations
    int64_t narrow_max = 4096;       // BFS frontiers of up to this many slots run in one workgroup (0: never)
    int64_t medium_max = 65536;      // ... up to this many in one cooperative launch of a few workgroups
    int32_t rn_limit = 2048;         // worklists of up to this many vertices run rounds in one workgroup
    bool bfs_cap = true;             // solve relabels stop once every vertex with excess has a height
    int32_t medium_blocks = 16;      //     of this many 1024-thread blocks (0 where unsupported)
    struct MedBufs {                 // their per-workgroup queue segments (made before a solve)
        int4* q = nullptr;
        unsigned long long* rec = nullptr;
        int64_t seg = 0;
        int blocks = 0;
    };
    MedBufs med, med2;               // main lane, pull lane
    bool coop_ok = false;            // the device supports cooperative launch
    std::atomic<bool> coop_broken{false};  // a cooperative launch failed: multi-block levels only
                                     // (set by either lane of a push-pull repair)
    int cus = 256;                   // compute units of the device
    bool graph_capture = false;      // pipelined iterations replayed from a captured HIP graph
    bool capture_failed = false;     // capture or instantiation failed once: launch kernel by kernel
    bool no_capture = false;         // this call instantiates no new graph (allocation-free entry point)
    bool heights_exact = true;       // heights are the last relabel's BFS distances (else a valid labelling
                                     // left by the round that ended the solve)
    hipStream_t cap_stream = nullptr;  // stream the iteration is captured on (never launched on)
    struct ItGraph {
        std::vector<long long> key;  // what it was captured with
        hipGraphExec_t exec;
    };
    std::vector<ItGraph> it_graphs;  // captured pipelined iterations
    int32_t* halt_d = nullptr;       // the loop kernels' halt word (next to the slot count)
    long long* nslots_d = nullptr;   // the used slot count in device memory, then the halt word (kept
                                     // while offloaded)
    // incremental worklists between relabels (made on first use)
    int32_t* act_list = nullptr;   // vertices whose excess turned positive in a round
    int32_t* mark = nullptr;       // per vertex: the round that last listed it
    int32_t* wlb[3] = {nullptr, nullptr, nullptr};  // second set of degree-bin worklists
    int32_t epoch = 0;
    // parallel push-pull repair (Section 5.2, O2): the pull side's lane and
    // heights, made on first use
    int32_t push_pull = 0;
    hipStream_t stream2 = nullptr;
    int2* q2[2] = {nullptr, nullptr};
    int64_t q2_cap = 0;
    int32_t* wl2[3] = {nullptr, nullptr, nullptr};
    mf::GrBits bits2{};
    DevCounters* ctr2 = nullptr;
    DevCounters* ctr2_h = nullptr;  // pinned
    int32_t* h2 = nullptr;
    // while offloaded the state lives in these pinned host buffers (kept for
    // the next offload) and the device holds only the counters
    bool offloaded = false;
    struct HostCopy {
        int2* cr = nullptr;
        int32_t *rev = nullptr, *cap = nullptr, *capsum = nullptr;
        int32_t *row_ptr = nullptr, *row_len = nullptr, *row_sorted = nullptr, *h = nullptr;
        int64_t* e = nullptr;
        int64_t slots = 0;
    } hc;
};

namespace mf {

mf_status resolve_tuning(const mf_options& o, Tuning* t) {
    Tuning r{};
    r.kc_option = o.kernel_cycles > 0 ? o.kernel_cycles : 0;
    r.gr = GrTune{GR_BU_ALPHA, GR_BU_BETA, GR_STAGE_MIN, 0, 0, 0};
    r.round_div = 4;
    if (o.bfs_stage_min > 0) r.gr.stage_min = o.bfs_stage_min;
    if (o.bfs_bottom_up < 0 || o.bfs_bottom_up > 2) return MF_ERR_INVALID;
    r.gr.bu_wide = o.bfs_bottom_up == 1;
    r.gr.bu_lb = o.bfs_bottom_up == 2;
    r.long_cycles = 1;
    if (o.long_row_cycles > 0) r.long_cycles = o.long_row_cycles;
    if (o.bfs_alpha > 0) r.gr.bu_alpha = o.bfs_alpha;
    if (o.bfs_alpha < 0) r.gr.bu_alpha = 0;
    if (o.bfs_beta > 0) r.gr.bu_beta = o.bfs_beta;
    if (o.round_div > 0) r.round_div = o.round_div;
    r.bin0 = o.bin_thread_max > 0 ? o.bin_thread_max : BIN0_MAX;
    r.bin1 = o.bin_wave_max > 0 ? o.bin_wave_max : BIN1_MAX;
    if (r.bin1 < r.bin0) return MF_ERR_INVALID;
    r.batch_block = o.batch_block == 0 ? 1024 : o.batch_block;
    if (r.batch_block != 256 && r.batch_block != 512 && r.batch_block != 1024) return MF_ERR_INVALID;
    *t = r;
    return MF_OK;
}

}  // namespace mf

namespace {

#define MF_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) {                        \
            g->poisoned = true;                        \
            return MF_ERR_DEVICE;                      \
        }                                              \
    } while (0)

template <class T>
hipError_t dalloc(mf_graph* g, T** p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    return g->mem.allocate((void**)p, bytes);
}

template <class T>
void dfree(mf_graph* g, T*& p) {
    g->mem.release((void*)p);
    p = nullptr;
}

// ---- per-kernel event timing ------------------------------------------------

hipEvent_t take_event(mf_graph* g) {
    if (!g->ev_pool.empty()) {
        hipEvent_t e = g->ev_pool.back();
        g->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

template <class F>
void timed(mf_graph* g, int cls, F&& launch) {
    if (!(g->prof_mask >> cls & 1u)) {
        launch();
        return;
    }
    hipEvent_t a = take_event(g), b = take_event(g);
    (void)hipEventRecord(a, g->stream);
    launch();
    (void)hipEventRecord(b, g->stream);
    g->ev_pending.push_back({cls, {a, b}});
}

// After the stream is synchronised: fold the recorded launches into totals.
void settle_events(mf_graph* g) {
    for (auto& p : g->ev_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            g->kernel_ms[p.first] += ms;
            g->kernel_launches[p.first]++;
        }
        g->ev_pool.push_back(p.second.first);
        g->ev_pool.push_back(p.second.second);
    }
    g->ev_pending.clear();
}

// Profiled calls: sum the kernels' per-block byte partials (one small
// kernel), read them back and add the selected classes to the totals.
void fold_bytes(mf_graph* g) {
    if (!g->prof_mask) return;
    mf::launch_reduce_bytes(g->dg, g->ctr, g->stream);
    if (hipMemcpyAsync(g->ctr_h, g->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
        hipStreamSynchronize(g->stream) != hipSuccess)
        return;
    for (int c = 0; c < 8; ++c)
        if (g->prof_mask >> c & 1u) g->kernel_bytes[c] += (double)g->ctr_h->bytes[c];
}

mf_status read_counters(mf_graph* g) {
    MF_HIP(hipMemcpyAsync(g->ctr_h, g->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, g->stream));
    MF_HIP(hipStreamSynchronize(g->stream));
    return MF_OK;
}

void free_structure(mf_graph* g) {
    dfree(g, g->dg.row_ptr);
    dfree(g, g->dg.row_len);
    dfree(g, g->dg.row_sorted);
    dfree(g, g->dg.cr);
    dfree(g, g->dg.rev);
    dfree(g, g->dg.cap);
    dfree(g, g->dg.capsum);
    dfree(g, g->win);
    dfree(g, g->q[0]);
    dfree(g, g->q[1]);
}

void free_round_lists(mf_graph* g) {
    dfree(g, g->dg.h_prev);
    dfree(g, g->act_list);
    dfree(g, g->mark);
    for (auto& w : g->wlb) dfree(g, w);
    g->epoch = 0;
}

void free_med(mf_graph* g, mf_graph::MedBufs& mb) {
    dfree(g, mb.q);
    dfree(g, mb.rec);
    mb.seg = 0;
    mb.blocks = 0;
}

void free_lane2(mf_graph* g) {
    free_round_lists(g);
    free_med(g, g->med2);
    dfree(g, g->q2[0]);
    dfree(g, g->q2[1]);
    g->q2_cap = 0;
    for (auto& w : g->wl2) dfree(g, w);
    dfree(g, g->bits2.visited);
    g->bits2.fb = nullptr;
    dfree(g, g->ctr2);
    dfree(g, g->h2);
}

void free_all(mf_graph* g) {
    if (!g->it_graphs.empty()) (void)hipStreamSynchronize(g->stream);
    for (auto& ig : g->it_graphs) (void)hipGraphExecDestroy(ig.exec);
    g->it_graphs.clear();
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
    free_lane2(g);
    free_med(g, g->med);
    if (g->ctr2_h) (void)hipHostFree(g->ctr2_h);
    g->ctr2_h = nullptr;
    free_structure(g);
    dfree(g, g->dg.e);
    dfree(g, g->dg.h);
    for (auto& w : g->wl) dfree(g, w);
    dfree(g, g->ctr);
    dfree(g, g->nslots_d);
    if (g->ctr_h) (void)hipHostFree(g->ctr_h);
    g->ctr_h = nullptr;
    dfree(g, g->need);
    dfree(g, g->slot_of);
    dfree(g, g->touched);
    dfree(g, g->upd);
    if (g->upd_h) (void)hipHostFree(g->upd_h);
    g->upd_h = nullptr;
    g->upd_h_dev = nullptr;
    dfree(g, g->tb.key);
    dfree(g, g->tb.win);
    dfree(g, g->tb.slot);
    dfree(g, g->side);
    dfree(g, g->cut_acc);
    dfree(g, g->bits.visited);
    dfree(g, g->dg.bytes_part);
    for (auto& p : g->ev_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (auto e : g->ev_pool) (void)hipEventDestroy(e);
    g->ev_pending.clear();
    g->ev_pool.clear();
    for (int k = 0; k < 2; ++k) {
        if (g->snap_ev[k]) (void)hipEventSynchronize(g->snap_ev[k]);
        if (g->snap_ev[k]) (void)hipEventDestroy(g->snap_ev[k]);
        if (g->snap_h[k]) (void)hipHostFree(g->snap_h[k]);
        g->snap_ev[k] = nullptr;
        g->snap_h[k] = nullptr;
    }
}

// Pinned counter snapshots and their events for pipelined iterations.
mf_status ensure_snapshots(mf_graph* g) {
    for (int k = 0; k < 2; ++k) {
        if (!g->snap_h[k] && hipHostMalloc((void**)&g->snap_h[k], sizeof(DevCounters), hipHostMallocDefault) != hipSuccess)
            return MF_ERR_OUT_OF_MEMORY;
        if (!g->snap_ev[k] && hipEventCreateWithFlags(&g->snap_ev[k], hipEventDisableTiming) != hipSuccess)
            return MF_ERR_DEVICE;
    }
    return MF_OK;
}

// Allocate and upload the slot arrays of a Bi-CSR (plus the arrays whose size
// follows the slot count).  res_init: residuals to upload, or empty for
// res = cap (zero flow).
mf_status upload_structure(mf_graph* g, const mf::HostBiCSR& b, const std::vector<int32_t>& res_init) {
    const int32_t n = g->n;
    const int64_t S = b.row_ptr[(size_t)n];
    if (dalloc(g, &g->dg.row_ptr, n + 1) != hipSuccess || dalloc(g, &g->dg.row_len, n) != hipSuccess ||
        dalloc(g, &g->dg.row_sorted, n) != hipSuccess || dalloc(g, &g->dg.cr, S) != hipSuccess ||
        dalloc(g, &g->dg.rev, S) != hipSuccess || dalloc(g, &g->dg.cap, S) != hipSuccess ||
        dalloc(g, &g->dg.capsum, S) != hipSuccess ||
        dalloc(g, &g->win, S) != hipSuccess)
        return MF_ERR_OUT_OF_MEMORY;
    g->q_cap = (int64_t)n + S / mf::GR_CHUNK + 64;
    if (dalloc(g, &g->q[0], g->q_cap) != hipSuccess || dalloc(g, &g->q[1], g->q_cap) != hipSuccess)
        return MF_ERR_OUT_OF_MEMORY;
    std::vector<int2> cr((size_t)S);
    std::vector<int32_t> capsum((size_t)S, 0);
    for (int64_t j = 0; j < S; ++j) {
        cr[(size_t)j] = make_int2(b.col[(size_t)j], res_init.empty() ? b.cap[(size_t)j] : res_init[(size_t)j]);
        if (b.rev[(size_t)j] >= 0) capsum[(size_t)j] = b.cap[(size_t)j] + b.cap[(size_t)b.rev[(size_t)j]];
    }
    hipStream_t st = g->stream;
    MF_HIP(hipMemcpyAsync(g->dg.row_ptr, b.row_ptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.row_len, b.row_len.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.row_sorted, b.row_sorted.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.cr, cr.data(), sizeof(int2) * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.rev, b.rev.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.cap, b.cap.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.capsum, capsum.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, st));
    mf::launch_fill_i32(g->win, -1, S, st);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(st));  // host vectors die on return
    g->slot_cap = S;
    return MF_OK;
}

void free_host_copy(mf_graph* g) {
    mf_graph::HostCopy& c = g->hc;
    void* bufs[] = {c.cr, c.rev, c.cap, c.capsum, c.row_ptr, c.row_len, c.row_sorted, c.h, c.e};
    for (void* p : bufs)
        if (p) (void)hipHostFree(p);
    c = mf_graph::HostCopy{};
}

template <class T>
hipError_t halloc(T** p, int64_t count) {
    return hipHostMalloc((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1), hipHostMallocDefault);
}

// Every device buffer except the counters (the state is elsewhere by then).
void free_device_state(mf_graph* g) {
    free_lane2(g);
    free_med(g, g->med);
    free_structure(g);
    dfree(g, g->dg.e);
    dfree(g, g->dg.h);
    for (auto& w : g->wl) dfree(g, w);
    dfree(g, g->need);
    dfree(g, g->slot_of);
    dfree(g, g->touched);
    dfree(g, g->upd);
    if (g->upd_h) (void)hipHostFree(g->upd_h);
    g->upd_h = nullptr;
    g->upd_h_dev = nullptr;
    dfree(g, g->tb.key);
    dfree(g, g->tb.win);
    dfree(g, g->tb.slot);
    dfree(g, g->side);
    dfree(g, g->cut_acc);
    dfree(g, g->bits.visited);
    g->bits.fb = nullptr;
    dfree(g, g->dg.bytes_part);
    g->k_cap = 0;
    g->tb.capacity = 0;
}

// Tuning fields of a handle from resolved options; KC defaults to round(m/n)
// (at least 1).  The LDS-staging flag is the device's and stays.
void apply_tuning(mf_graph* g, const mf::Tuning& t) {
    int64_t kc = t.kc_option > 0 ? t.kc_option : (g->m_unique + g->n / 2) / g->n;
    g->kc = (int32_t)std::max<int64_t>(1, kc);
    int lds = g->tune.lds;
    g->tune = t.gr;
    g->tune.lds = lds;
    g->round_div = t.round_div;
    g->dg.bin0_max = t.bin0;
    g->dg.bin1_max = t.bin1;
    g->kc_block = t.long_cycles;
}

// Loop and relabel settings of a handle from its options (0 = default).
void apply_loop_options(mf_graph* g, const mf_options& o) {
    auto on = [](int32_t v, bool dflt) { return v > 0 ? true : v < 0 ? false : dflt; };
    g->first_chunk = o.bfs_first_chunk > 0 ? o.bfs_first_chunk : 7;
    g->narrow_max = o.bfs_narrow_slots < 0 ? 0 : o.bfs_narrow_slots > 0 ? o.bfs_narrow_slots : 4096;
    g->medium_max = o.bfs_medium_slots < 0 ? 0 : o.bfs_medium_slots > 0 ? o.bfs_medium_slots : 65536;
    g->medium_blocks = o.bfs_medium_blocks > 0 ? o.bfs_medium_blocks : 16;
    // mid-size frontiers need cooperative launch (every block resident)
    if (!g->coop_ok || g->medium_max <= g->narrow_max) g->medium_blocks = 0;
    g->gr_grid = o.bfs_level_blocks > 0 ? o.bfs_level_blocks : std::max(32, g->cus * 4);
    g->tune.lds = on(o.bfs_lds_bitmap, false) && mf::gr_level_lds_bytes(g->bits.nwords, g->device) > 0 ? 1 : 0;
    g->round_min = o.round_min > 0 ? o.round_min : 2;
    g->round_max = o.round_max > 0 ? o.round_max : 4096;
    g->rn_limit = o.round_narrow < 0 ? 0 : o.round_narrow > 0 ? o.round_narrow : 2048;
    g->bfs_cap = on(o.bfs_cap, true);
    g->incremental_rounds = !on(o.round_scan, false);
    g->queue_rounds = on(o.queue_rounds, true);
    g->pipeline = on(o.pipeline, true);
    g->graph_capture = on(o.graph_capture, false);
    g->trace_gr = on(o.trace, false);
}

// Push/relabel cycles per launch for worklist bin b (2: rows a workgroup takes).
int32_t kc_for_bin(const mf_graph* g, int b) { return b == 2 ? std::min(g->kc, g->kc_block) : g->kc; }

mf_status ensure_batch_capacity(mf_graph* g, int64_t k) {
    if (k <= g->k_cap) return MF_OK;
    int64_t cap = std::max<int64_t>(k, 1024);
    int32_t tcap = 64;
    while (tcap < 2 * cap) tcap *= 2;
    MF_HIP(hipStreamSynchronize(g->stream));
    dfree(g, g->slot_of);
    dfree(g, g->touched);
    dfree(g, g->upd);
    dfree(g, g->tb.key);
    dfree(g, g->tb.win);
    dfree(g, g->tb.slot);
    if (g->upd_h) (void)hipHostFree(g->upd_h);
    g->upd_h = nullptr;
    g->upd_h_dev = nullptr;
    if (hipHostMalloc((void**)&g->upd_h, sizeof(mf_update) * (size_t)cap, hipHostMallocDefault) != hipSuccess) {
        g->upd_h = nullptr;
        g->k_cap = 0;
        return MF_ERR_OUT_OF_MEMORY;
    }
    // its address for kernels (pinned host memory is mapped into the device's
    // address space); without one the batch goes by hipMemcpyAsync
    g->upd_h_dev = nullptr;
    if (hipHostGetDevicePointer((void**)&g->upd_h_dev, g->upd_h, 0) != hipSuccess) {
        (void)hipGetLastError();
        g->upd_h_dev = nullptr;
    }
    if (dalloc(g, &g->slot_of, cap) != hipSuccess || dalloc(g, &g->touched, cap) != hipSuccess ||
        dalloc(g, &g->upd, cap) != hipSuccess || dalloc(g, &g->tb.key, tcap) != hipSuccess ||
        dalloc(g, &g->tb.win, 2 * (int64_t)tcap) != hipSuccess ||
        dalloc(g, &g->tb.slot, 2 * (int64_t)tcap) != hipSuccess) {
        g->k_cap = 0;
        return MF_ERR_OUT_OF_MEMORY;
    }
    g->tb.capacity = tcap;
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->tb.key), -1, 2 * (int64_t)tcap, g->stream);
    mf::launch_fill_i32(g->tb.win, -1, 2 * (int64_t)tcap, g->stream);
    MF_HIP(hipGetLastError());
    g->k_cap = cap;
    return MF_OK;
}

// ---- the push-relabel loop ----------------------------------------------------

// What one loop runs on.  The solve: backward BFS from t with deficits as
// extra sinks, positive-excess worklist, push-relabel and remove-invalid-
// edges.  Completing a preflow into a flow reuses the loop twice on a copy of
// the state: pushes toward s (root s, t pinned), then pulls from t (forward
// BFS, negative-excess worklist, s pinned).
// The scratch one loop runs on: a stream, BFS queues, worklists, bitmaps and
// counters.  The handle's own lane is the main one (timed when profiling);
// the parallel push-pull repair runs a second lane on a stream of its own.
struct Lane {
    hipStream_t stream = nullptr;
    int2* q[2] = {nullptr, nullptr};
    int32_t* wl[3] = {nullptr, nullptr, nullptr};
    mf::GrBits bits{};
    DevCounters* ctr = nullptr;
    DevCounters* ctr_h = nullptr;
    mf::MedQueue mq{};      // mid-size levels' segments (mq.q null: none, multi-block levels instead)
    int mq_blocks = 0;
    bool main = true;
};

void set_med(Lane& L, const mf_graph::MedBufs& mb) {
    L.mq = mf::MedQueue{mb.q, mb.rec, mb.seg};
    L.mq_blocks = mb.blocks;
}

Lane main_lane(mf_graph* g) {
    Lane L;
    L.stream = g->stream;
    L.q[0] = g->q[0];
    L.q[1] = g->q[1];
    for (int b = 0; b < 3; ++b) L.wl[b] = g->wl[b];
    L.bits = g->bits;
    L.ctr = g->ctr;
    L.ctr_h = g->ctr_h;
    set_med(L, g->med);
    return L;
}

struct LoopMode {
    DevGraph dg;
    Lane L;
    int seed_deficits = 1;
    bool forward = false;
    int sign = 1;
    bool pull = false;
    bool rie = true;
    bool topology = false;
};

LoopMode solve_mode(mf_graph* g) {
    LoopMode m;
    m.dg = g->dg;
    m.L = main_lane(g);
    m.topology = g->opt.topology_driven != 0;
    return m;
}

// Event timing on the main lane only (the host bookkeeping is not shared
// across threads).
template <class F>
void timed(mf_graph* g, const Lane& L, int cls, F&& launch) {
    if (L.main) timed(g, cls, launch);
    else launch();
}

mf_status read_lane(mf_graph* g, const Lane& L) {
    MF_HIP(hipMemcpyAsync(L.ctr_h, L.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, L.stream));
    MF_HIP(hipStreamSynchronize(L.stream));
    return MF_OK;
}

// Global relabel: seeds, then levels in growing chunks; each level launch
// reads the frontier size on the device, so the host checks only after a
// chunk.  Returns the number of level launches.
//
// tail (optional): launches queued right behind the first multi-block chunk,
// before the host reads the counters -- the guarded worklist build and the
// rounds after it.  *tail_valid tells whether the BFS ended within that
// chunk, i.e. whether the tail did its work (else it was a no-op).
mf_status global_relabel(mf_graph* g, const LoopMode& m, int64_t* levels_out, int* depth_out,
                         const std::function<void(int)>* tail = nullptr, bool* tail_valid = nullptr) {
    // *levels_out counts level launches (a chunk's last ones may find the BFS
    // over); *depth_out is the BFS's depth as the level kernels recorded it.
    // The seed and depth hints kept on the handle are the main lane's (the
    // pull lane of a push-pull repair runs on another thread).
    hipStream_t st = m.L.stream;
    bool tail_queued = false;
    if (tail_valid) *tail_valid = false;
    timed(g, m.L, mf::KC_GRS, [&] { mf::launch_gr_init(m.dg, m.L.q[0], m.L.ctr, m.L.bits, m.seed_deficits, st); });
    int level = 0;
    // the first chunk covers the last relabel's depth, so that a tail queued
    // behind it usually finds the BFS over
    int chunk = g->trace_gr ? 1 : (tail ? std::min(64, std::max(g->first_chunk, g->last_depth + 1)) : g->first_chunk);
    const bool main = m.L.main;
    // thin frontiers run in one workgroup, several levels per launch; the
    // first frontier is tried that way, later ones when a chunk leaves one
    // small enough
    bool narrow = g->narrow_max > 0 && !g->trace_gr && (g->narrow_seed || !m.L.main);
    bool medium = false;  // set when a read finds a mid-size frontier waiting
    const int64_t medium_cap = std::min<int64_t>(g->medium_max, m.L.mq.seg);
    const int medium_grid = std::min<int>(g->medium_blocks, m.L.mq_blocks);
    auto mid_size = [&](int lv) {
        const int64_t slots = (int64_t)(m.L.ctr_h->front[lv % 3] >> 32);
        return medium_grid > 0 && m.L.mq.q && !g->coop_broken && !g->trace_gr && slots > g->narrow_max &&
               slots <= medium_cap;
    };
    auto t_last = std::chrono::steady_clock::now();
    if (g->trace_gr) {
        mf_status rc = read_lane(g, m.L);
        if (rc != MF_OK) return rc;
        const unsigned long long f = m.L.ctr_h->front[0];
        std::fprintf(stderr, "[gr] seeds %u slots %llu\n", (unsigned)(f & 0xFFFFFFFFull), f >> 32);
        t_last = std::chrono::steady_clock::now();
    }
    for (;;) {
        if (narrow) {
            timed(g, m.L, mf::KC_GRS, [&] {
                mf::launch_gr_narrow(m.dg, level, m.L.q[0], m.L.q[1], m.L.ctr, m.L.bits, g->narrow_max, m.forward,
                                     st);
            });
            MF_HIP(hipGetLastError());
            mf_status rc = read_lane(g, m.L);
            if (rc != MF_OK) return rc;
            const int level_before = level;
            level = m.L.ctr_h->levels;
            if (level_before == 0 && main)
                g->narrow_seed = (int64_t)(m.L.ctr_h->seed_front >> 32) <= g->narrow_max;
            const int cnt = (int)(unsigned)(m.L.ctr_h->front[level % 3] & 0xFFFFFFFFull);
            if (cnt == 0) break;
            if (level > g->n + 2) {
                g->poisoned = true;
                return MF_ERR_DEVICE;  // a BFS cannot have more than n levels
            }
            // the multi-block levels read the current frontier's bitmap (the
            // one-workgroup levels do not keep it; untouched if none ran)
            if (level != level_before)
                timed(g, m.L, mf::KC_GRS,
                      [&] { mf::launch_frontier_bitmap(m.L.q[level & 1], cnt, m.L.bits, level, st); });
            chunk = g->first_chunk;
            medium = mid_size(level);
        }
        if (medium) {
            hipError_t err = hipSuccess;
            timed(g, m.L, mf::KC_GRS, [&] {
                err = mf::launch_gr_medium(m.dg, level, m.L.q[0], m.L.q[1], m.L.ctr, m.L.bits, g->tune,
                                           medium_cap, m.forward, medium_grid, m.L.mq, st);
            });
            if (err != hipSuccess) {
                (void)hipGetLastError();
                g->coop_broken = true;  // no cooperative launch here: multi-block levels only
            } else {
                mf_status rc = read_lane(g, m.L);
                if (rc != MF_OK) return rc;
                if (m.L.ctr_h->bar_err) {
                    g->poisoned = true;
                    return MF_ERR_DEVICE;
                }
                const int level_before = level;
                level = m.L.ctr_h->levels;
                const int cnt = (int)(unsigned)(m.L.ctr_h->front[level % 3] & 0xFFFFFFFFull);
                if (cnt == 0) break;
                if (level > g->n + 2) {
                    g->poisoned = true;
                    return MF_ERR_DEVICE;  // a BFS cannot have more than n levels
                }
                // the multi-block levels read the current frontier's bitmap,
                // which the mid-size levels do not keep
                if (level != level_before)
                    timed(g, m.L, mf::KC_GRS,
                          [&] { mf::launch_frontier_bitmap(m.L.q[level & 1], cnt, m.L.bits, level, st); });
                chunk = g->first_chunk;
            }
            medium = false;  // a larger frontier waits: multi-block levels
        }
        for (int i = 0; i < chunk; ++i, ++level)
            timed(g, m.L, mf::KC_GR, [&] {
                mf::launch_gr_level(m.dg, level, m.L.q[level & 1], m.L.q[(level + 1) & 1], m.L.ctr,
                                    m.L.bits, g->tune, g->gr_grid, m.forward, st);
            });
        const bool tail_now = tail && !tail_queued;
        if (tail_now) {
            (*tail)(level);
            tail_queued = true;
        }
        MF_HIP(hipGetLastError());
        mf_status rc = read_lane(g, m.L);
        if (rc != MF_OK) return rc;
        // seeds of the next relabel: like this one's, as its level 0 recorded them
        if (main) g->narrow_seed = (int64_t)(m.L.ctr_h->seed_front >> 32) <= g->narrow_max;
        const int cnt = (int)(unsigned)(m.L.ctr_h->front[level % 3] & 0xFFFFFFFFull);
        if (g->trace_gr) {
            // the level just done: its frontier, the unvisited slots before it,
            // the direction rule's choice, its next frontier, host wall time
            const DevCounters& c = *m.L.ctr_h;
            const int lv = level - 1;
            const unsigned long long f = c.front[lv % 3];
            const long long fs = (long long)(f >> 32), cin = (long long)(f & 0xFFFFFFFFull);
            const long long mu = c.unv[lv % 3];
            const bool bu = g->tune.bu_alpha > 0 && fs * g->tune.bu_alpha > mu && cin * g->tune.bu_beta > g->n;
            const auto now = std::chrono::steady_clock::now();
            std::fprintf(stderr, "[gr] level %d frontier %lld slots %lld unvisited %lld %s next %d us %.1f\n", lv,
                         cin, fs, mu, bu ? "bu" : "td", cnt,
                         std::chrono::duration<double, std::micro>(now - t_last).count());
            t_last = now;
        }
        if (cnt == 0) {
            if (tail_now && tail_valid) *tail_valid = true;
            break;
        }
        if (level > g->n + 2) {
            g->poisoned = true;
            return MF_ERR_DEVICE;  // a BFS cannot have more than n levels
        }
        if (g->trace_gr) continue;  // one level per launch
        chunk = std::min(chunk * 2, 64);
        narrow = g->narrow_max > 0 && (int64_t)(m.L.ctr_h->front[level % 3] >> 32) <= g->narrow_max;
        medium = !narrow && mid_size(level);
    }
    *levels_out += level;
    *depth_out = m.L.ctr_h->levels;
    if (main) g->last_depth = *depth_out;
    return MF_OK;
}

// Global relabel followed by the worklist build (and value), leaving the
// counters in ctr_h.  With cooperative launch support this is one persistent
// kernel (every BFS level behind a grid barrier); otherwise one launch per
// level plus one for the worklist.
mf_status relabel_and_worklist(mf_graph* g, const LoopMode& m, int64_t* levels, int* depth,
                               const std::function<void(int)>* tail = nullptr, bool* tail_valid = nullptr) {
    hipStream_t st = m.L.stream;
    if (g->persistent_grid > 0) {
        hipError_t err = hipSuccess;
        timed(g, m.L, mf::KC_GR, [&] {
            err = mf::launch_gr_persistent(m.dg, m.L.q[0], m.L.q[1], m.L.ctr, m.L.bits, g->tune, m.seed_deficits,
                                           m.forward, m.L.wl[0], m.L.wl[1], m.L.wl[2], m.topology, m.sign,
                                           g->persistent_grid, st);
        });
        MF_HIP(err);
        mf_status rc = read_lane(g, m.L);
        if (rc != MF_OK) return rc;
        if (m.L.ctr_h->bar_err) {
            g->poisoned = true;
            return MF_ERR_DEVICE;
        }
        *levels += m.L.ctr_h->levels;
        *depth = m.L.ctr_h->levels;
        return MF_OK;
    }
    mf_status rc = global_relabel(g, m, levels, depth, tail, tail_valid);
    if (rc != MF_OK) return rc;
    if (tail_valid && *tail_valid) return MF_OK;  // the tail built the worklist; counters read
    timed(g, m.L, mf::KC_WL, [&] {
        mf::launch_build_worklist(m.dg, m.L.wl[0], m.L.wl[1], m.L.wl[2], m.L.ctr, m.topology, m.sign, st);
    });
    MF_HIP(hipGetLastError());
    return read_lane(g, m.L);
}

// Loop {global relabel; worklist; stop if no active vertex; R rounds of
// push-relabel, remove invalid edges and worklist on the current heights}.
// The stop test that ends the loop is taken right after a fresh global
// relabel, so at exit A = {h = |V|} is a cut whose capacity is the value.
// Between relabels the heights stay a valid labelling (push-relabel lifts by
// the lowest neighbour + 1, remove-invalid-edges saturates every steep
// residual slot), so further rounds need no relabel; a vertex activated by a
// push waits for the next worklist, so each round moves excess about one
// more hop.  R is the relabel's depth divided by round_div, at least
// round_min (2): a deep BFS (long augmenting paths) buys many cheap rounds; on
// a shallow one (RMAT, random graphs: depth under 10) a second round, which
// starts from the activations of the first instead of a scan, still costs
// well under a relabel and saves about a third of them.
//
// One round: push-relabel (two launches) and remove-invalid-edges (one).
// dev: the bins' sizes are the worklist counts on the device when the
// kernels run, cnt[] only upper bounds for their grids.
mf_status push_round(mf_graph* g, const LoopMode& m, int32_t* const wl[3], const int cnt[3], bool dev = false) {
    hipStream_t st = m.L.stream;
    const int32_t* dcount = dev ? m.L.ctr->wl : nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    timed(g, m.L, mf::KC_PR, [&] {
        mf::launch_push_relabel_round(m.dg, wl, cnt, kc_for_bin(g, 0), kc_for_bin(g, 2), m.pull, st, dcount);
    });
    if (g->trace_gr) {
        MF_HIP(hipStreamSynchronize(st));
        std::fprintf(stderr, "[loop]   push rows by bin %d %d %d us %.1f\n", cnt[0], cnt[1], cnt[2],
                     std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count());
    }
    if (m.rie) timed(g, m.L, mf::KC_RIE, [&] { mf::launch_remove_invalid_round(m.dg, wl, cnt, m.L.ctr, st, dcount); });
    MF_HIP(hipGetLastError());
    return MF_OK;
}

// The mid-size levels' segments for the handle's settings: each workgroup
// appends at most one entry per slot it scans, and those levels scan at most
// medium_max slots (and fewer than the global queue holds; larger frontiers
// than MED_MAX_SEG slots go to the multi-block levels).
mf_status ensure_med(mf_graph* g, mf_graph::MedBufs& mb) {
    const int blocks = std::min(g->medium_blocks, mf::MED_MAX_BLOCKS);
    const int64_t seg = std::min<int64_t>(std::min<int64_t>(g->medium_max, g->q_cap), mf::MED_MAX_SEG);
    if (blocks <= 0 || seg <= 0) {
        free_med(g, mb);
        return MF_OK;
    }
    if (mb.q && mb.blocks >= blocks && mb.seg >= seg) return MF_OK;
    free_med(g, mb);
    if (dalloc(g, &mb.q, 2 * (int64_t)blocks * seg) != hipSuccess || dalloc(g, &mb.rec, 3 * (int64_t)blocks) != hipSuccess) {
        free_med(g, mb);
        return MF_ERR_OUT_OF_MEMORY;
    }
    mb.seg = seg;
    mb.blocks = blocks;
    return MF_OK;
}

// Buffers of the incremental worklists between relabels.
mf_status ensure_round_lists(mf_graph* g) {
    if (g->act_list) return MF_OK;
    const int64_t n = g->n;
    if (dalloc(g, &g->act_list, n) != hipSuccess || dalloc(g, &g->mark, n + 1) != hipSuccess ||
        dalloc(g, &g->wlb[0], n) != hipSuccess || dalloc(g, &g->wlb[1], n) != hipSuccess ||
        dalloc(g, &g->wlb[2], n) != hipSuccess) {
        free_round_lists(g);
        return MF_ERR_OUT_OF_MEMORY;
    }
    mf::launch_fill_i32(g->mark, 0, n + 1, g->stream);
    g->epoch = 0;
    MF_HIP(hipGetLastError());
    return MF_OK;
}

// Iterations are pipelined while the last relabel was shallower than this
// (at most two rounds per relabel).
constexpr int PIPELINE_DEPTH = 16;

// Rounds on a worklist short enough for the one-workgroup round kernel cost
// a few microseconds each and stop as soon as the list empties: a relabel
// whose worklist is that thin buys at least this many of them before the
// next relabel (deep BFS on grids ends with many shallow relabels).
constexpr int THIN_ROUNDS_MIN = 8;

// The next-worklist marks compare with an epoch word in device memory
// (mark[n]) that every next-worklist build moves on by one before it runs.
// The host counts the builds it queues; before the word could wrap it clears
// every mark and the word (stale marks of an old epoch only ever cost a
// vertex one round's delay: the loop stops on a full scan after a relabel).
void count_epochs(mf_graph* g, hipStream_t st, int builds) {
    if (g->epoch > INT_MAX - 1024 - builds) {
        mf::launch_fill_i32(g->mark, 0, (int64_t)g->n + 1, st);
        g->epoch = 0;
    }
    g->epoch += builds;
}

// Everything a captured pipelined iteration bakes into its launches: the
// graph and lane buffers, the loop mode, the tuning and the chunk.  The slot
// count is left out (the relabel reads it from device memory).
std::vector<long long> capture_key(const mf_graph* g, const LoopMode& m, const LoopMode& qm, int C) {
    std::vector<long long> k;
    auto P = [&](const void* p) { k.push_back((long long)(intptr_t)p); };
    for (const DevGraph* d : {&m.dg, &qm.dg}) {
        k.insert(k.end(), {d->n, d->s, d->t, d->root, d->pinned, d->count_bytes, d->bin0_max, d->bin1_max,
                           d->side_keep, d->act_cap});
        for (const void* p : {(const void*)d->row_ptr, (const void*)d->row_len, (const void*)d->row_sorted,
                              (const void*)d->cr, (const void*)d->rev, (const void*)d->cap, (const void*)d->capsum,
                              (const void*)d->e, (const void*)d->h, (const void*)d->nslots,
                              (const void*)d->bytes_part, (const void*)d->side, (const void*)d->act,
                              (const void*)d->act_cnt, (const void*)d->relab, (const void*)d->h_prev})
            P(p);
        k.push_back(d->bfs_cap);
    }
    const Lane& L = m.L;
    for (const void* p : {(const void*)L.q[0], (const void*)L.q[1], (const void*)L.wl[0], (const void*)L.wl[1],
                          (const void*)L.wl[2], (const void*)L.bits.visited, (const void*)L.bits.fb,
                          (const void*)L.ctr, (const void*)g->mark, (const void*)g->wlb[0], (const void*)g->wlb[1],
                          (const void*)g->wlb[2]})
        P(p);
    const mf::GrTune& t = g->tune;
    k.insert(k.end(), {L.bits.nwords, t.bu_alpha, t.bu_beta, t.stage_min, t.lds, t.bu_lb, t.bu_wide, g->gr_grid,
                       kc_for_bin(g, 0), kc_for_bin(g, 2), C, m.seed_deficits, m.sign, m.forward, m.topology,
                       m.pull, m.rie, qm.rie});
    return k;
}

// The pipelined iteration of chunk C as an instantiated HIP graph: captured
// on the handle's capture stream the first time, and again whenever
// something it bakes in changed (a relayout, a restore, new tuning); the
// last eight captures are kept (chunks follow the BFS depth, which varies a
// little).  Consecutive iterations use two instantiations (`copy` 0 and 1),
// so that queuing the next one never waits for the launch of the same
// executable still in flight.  nullptr when capture is unavailable: the
// caller launches the kernels one by one.
template <class F>
hipGraphExec_t iteration_graph(mf_graph* g, const LoopMode& m, const LoopMode& qm, int C, int copy, F&& enqueue) {
    std::vector<long long> key = capture_key(g, m, qm, C);
    key.push_back(copy);
    for (auto& ig : g->it_graphs)
        if (ig.key == key) return ig.exec;
    if (g->capture_failed || g->no_capture) return nullptr;
    if (g->it_graphs.size() >= 8) {
        // the oldest capture goes (it may still be running on the stream)
        if (hipStreamSynchronize(g->stream) != hipSuccess) return nullptr;
        (void)hipGraphExecDestroy(g->it_graphs.front().exec);
        g->it_graphs.erase(g->it_graphs.begin());
    }
    if (!g->cap_stream && hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        g->capture_failed = true;
        return nullptr;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    mf_status rc = MF_OK;
    hipError_t e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue(g->cap_stream);
        e = hipStreamEndCapture(g->cap_stream, &graph);
    }
    if (e == hipSuccess && rc == MF_OK && graph) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess || rc != MF_OK || !exec) {
        (void)hipGetLastError();
        if (exec) (void)hipGraphExecDestroy(exec);
        g->capture_failed = true;  // launch kernel by kernel from now on
        return nullptr;
    }
    g->it_graphs.push_back({std::move(key), exec});
    return exec;
}

mf_status run_loop(mf_graph* g, const LoopMode& m_in, int64_t* value) {
    LoopMode m = m_in;
    // every buffer a loop launches on must be set (a mode built by hand
    // without a lane would hand the kernels null pointers)
    const Lane& L = m.L;
    if (!L.stream || !L.q[0] || !L.q[1] || !L.wl[0] || !L.wl[1] || !L.wl[2] || !L.bits.visited ||
        !L.bits.fb || !L.ctr || !L.ctr_h || !m.dg.h || !m.dg.e || !m.dg.cr)
        return MF_ERR_INVALID;
    hipStream_t st = m.L.stream;
    int64_t iters = 0, levels = 0, active_sum = 0, rounds = 0, capped = 0;
    // The main lane queues the worklist build and the first two rounds right
    // behind the relabel's first chunk of BFS levels, sized on the device:
    // an iteration whose BFS ends within that chunk reads the counters back
    // once instead of three times.  (Rounds run on the worklist of a finished
    // relabel only: the build is guarded on the device.)
    const bool queue = g->queue_rounds && m.L.main && !m.pull && !m.topology && g->incremental_rounds &&
                       g->round_min >= 2 && !g->trace_gr && g->persistent_grid == 0;
    // The active set after a push-relabel plus remove-invalid-edges round is
    // taken under a valid labelling (the rounds keep h(u) <= h(v) + 1 on every
    // residual slot, Section 3.1; remove-invalid-edges repairs what races
    // broke).  While every sink -- t and each deficient vertex -- is at height
    // 0, a vertex at |V| cannot reach one (its height would have to fall by
    // |V| along a simple path), so an empty active set ends the loop there,
    // without another relabel, with the same value (the sinks' excess sum).
    // This is Algorithm 1's test after its kernels.  A vertex that remove-
    // invalid-edges made deficient sits at its own height: then the next
    // relabel decides, as before.  Heights at such an end are valid but not
    // exact distances: the cut is read after a fresh relabel (mf_min_cut).
    // Only the solve itself (sinks t and the deficits, remove-invalid-edges
    // on) ends this way.
    // (With push-pull the next repair reads the last cut from the heights:
    // those solves end after a relabel.)
    const bool shortcut =
        m.rie && !m.pull && m.sign == 1 && !m.forward && m.seed_deficits && m.L.main && !g->push_pull;
    // Optionally, the relabels of such a solve that follow a round (heights a
    // valid labelling) with every deficient vertex at height 0 stop once
    // every vertex with excess below |V| has its height (its BFS distance);
    // a vertex not reached by then keeps max(depth + 1, its old height) -- a
    // valid labelling (the kernels state why).  Excess that cannot reach a
    // sink (or a deficit above height 0) keeps the BFS going to its end, as
    // does the first relabel of every call.  Pushes only need a valid
    // labelling, and the loop's stop needs one too (A10); the cut is read
    // after an exact relabel.
    m.dg.bfs_cap = shortcut && g->bfs_cap && g->persistent_grid == 0 && m.dg.h_prev ? 1 : 0;
    if (m.dg.bfs_cap) mf::launch_set_i32(&m.L.ctr->lab_valid, 0, st);  // the first relabel runs to its end
    LoopMode qm = m;
    if (queue) {
        mf_status rc = ensure_round_lists(g);
        if (rc != MF_OK) return rc;
        qm.dg.act = g->act_list;
        qm.dg.act_cnt = &m.L.ctr->act;
        qm.dg.act_cap = g->n;
        // rounds right after a fresh relabel (whose heights are exact BFS
        // distances, a valid labelling): an out-slot can only turn steep at
        // a vertex whose height push-relabel raised, so remove-invalid-edges
        // visits just those rows.  The marks live in the first frontier
        // bitmap, free until the next relabel rewrites it.
        qm.dg.relab = m.L.bits.fb;
    }
    const int bounds[3] = {(int)g->n, (int)g->n, (int)g->n};
    mf_status tail_rc = MF_OK;
    // The launches queued behind the relabel's first chunk of levels on
    // stream `sm`'s lane: the guarded worklist build, the first round, the
    // second round's worklist from the first's (one next-worklist build: one
    // epoch), the second round.
    auto enqueue_tail = [&](const LoopMode& mm, const LoopMode& qq, int level_end) -> mf_status {
        hipStream_t s2 = mm.L.stream;
        timed(g, mm.L, mf::KC_WL, [&] {
            mf::launch_build_worklist(qq.dg, mm.L.wl[0], mm.L.wl[1], mm.L.wl[2], mm.L.ctr, mm.topology, mm.sign,
                                      s2, level_end);
        });
        // the build cleared the activation count; the next-worklist build
        // sets the worklist counts aside in wl_in (the host reads the
        // relabel's there), the second round keeps its own in wl
        mf_status rc = push_round(g, qq, mm.L.wl, bounds, true);
        timed(g, mm.L, mf::KC_WL, [&] {
            mf::launch_next_worklist(qq.dg, mm.L.wl, nullptr, g->wlb[0], g->wlb[1], g->wlb[2], g->mark,
                                     g->mark + g->n, mm.L.ctr, s2);
            // the first round left no active vertex: the value, and no second round
            if (shortcut) mf::launch_value_if_empty(qq.dg, mm.L.ctr, level_end, s2);
        });
        mf::launch_zero_act(mm.L.ctr, s2);
        if (rc == MF_OK) rc = push_round(g, qq, g->wlb, bounds, true);
        return rc;
    };
    const std::function<void(int)> tail = [&](int level_end) {
        count_epochs(g, st, 1);
        mf_status rc = enqueue_tail(m, qm, level_end);
        if (tail_rc == MF_OK) tail_rc = rc;
    };
    // Shallow relabels (depth under 16: at most two rounds each), no thin-
    // frontier start, no event timing: the next iteration -- relabel init,
    // its first chunk of levels, the queued tail and a copy of the counters
    // to a pinned snapshot -- is queued before the host waits for the
    // previous one's snapshot, so the device never idles on that read.  When
    // the previous iteration turns out to be the last (empty worklist), the
    // one queued behind it relabels the same residual graph to the same
    // heights and finds the same empty worklist: it changes nothing.  A BFS
    // that outlasts its chunk (or grows deep) sends the loop back to the
    // ordinary iterations below, which start with a fresh relabel.
    //
    // Every pipelined iteration launches the same kernels with the same
    // arguments (the chunk is fixed; the epoch and the slot count are read
    // from device memory), so by default the iteration is captured once
    // into a HIP graph and each later one is a single graph launch.
    bool finished = false;
    bool exact = false;  // the loop ended right after a relabel: heights are BFS distances
    if (queue && g->pipeline && !g->prof_mask && !g->narrow_seed && g->last_depth > 0 &&
        g->last_depth < PIPELINE_DEPTH) {
        mf_status rc = ensure_snapshots(g);
        if (rc != MF_OK) return rc;
        mf::launch_set_i32(g->halt_d, 0, st);
        // the relabel init, C levels, the tail and the halt test, on stream
        // s3 (st, or the capture stream)
        auto enqueue_iteration = [&](hipStream_t s3, int C) -> mf_status {
            LoopMode mm = m, qq = qm;
            mm.L.stream = qq.L.stream = s3;
            mf::launch_gr_init(mm.dg, mm.L.q[0], mm.L.ctr, mm.L.bits, mm.seed_deficits, s3);
            for (int lv = 0; lv < C; ++lv)
                mf::launch_gr_level(mm.dg, lv, mm.L.q[lv & 1], mm.L.q[(lv + 1) & 1], mm.L.ctr, mm.L.bits, g->tune,
                                    g->gr_grid, mm.forward, s3);
            mf_status r = enqueue_tail(mm, qq, C);
            mf::launch_halt_if_done(mm.L.ctr, C, shortcut, g->halt_d, s3);
            return r;
        };
        hipError_t queue_err = hipSuccess;
        auto queue_iteration = [&](int slot) -> int {
            // the first chunk covers the last relabel's depth
            const int C = std::min(64, std::max(g->first_chunk, g->last_depth + 1));
            hipGraphExec_t exec = nullptr;
            if (g->graph_capture)
                exec = iteration_graph(g, m, qm, C, slot,
                                       [&](hipStream_t s3) { return enqueue_iteration(s3, C); });
            count_epochs(g, st, 1);
            hipError_t e = hipSuccess;
            if (exec) {
                e = hipGraphLaunch(exec, st);
            } else {
                mf_status r2 = enqueue_iteration(st, C);
                if (tail_rc == MF_OK) tail_rc = r2;
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(g->snap_h[slot], m.L.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipEventRecord(g->snap_ev[slot], st);
            if (queue_err == hipSuccess) queue_err = e;
            return C;
        };
        int chunk[2];
        int k = 0;
        chunk[0] = queue_iteration(0);
        for (;;) {
            chunk[1 - k] = queue_iteration(1 - k);
            MF_HIP(hipGetLastError());
            MF_HIP(queue_err);
            if (tail_rc != MF_OK) return tail_rc;
            MF_HIP(hipEventSynchronize(g->snap_ev[k]));
            const DevCounters& c = *g->snap_h[k];
            levels += chunk[k];
            // the BFS outlasted the chunk: the tail did nothing
            if ((c.front[chunk[k] % 3] & 0xFFFFFFFFull) != 0) break;
            g->last_depth = c.levels;
            const int active = c.wl_in[3];  // the relabel's worklist (set aside before the second round's)
            active_sum += active;
            capped += c.bfs_capped != 0;
            if (active == 0) {
                *value = (int64_t)c.e_t + (int64_t)c.deficit_sum;
                *m.L.ctr_h = c;
                finished = true;
                exact = !c.bfs_capped;
                break;
            }
            if (shortcut && c.wl[3] == 0 && c.round_raised == 0) {  // the first round left no active vertex
                *value = (int64_t)c.round_e_t + (int64_t)c.round_deficit;
                *m.L.ctr_h = c;
                finished = true;
                ++iters;
                rounds += 1;
                break;
            }
            if (++iters > g->max_iter) {
                g->last_iterations = iters;
                mf::launch_set_i32(g->halt_d, 0, st);
                return MF_ERR_NOT_CONVERGED;
            }
            rounds += 2;
            if (g->last_depth >= PIPELINE_DEPTH) break;  // deep now: the ordinary loop runs more rounds per relabel
            k = 1 - k;
        }
        // leaving early: the iteration still queued runs to its end first
        // (it may have ended the loop and set the halt word: cleared below)
        if (!finished) MF_HIP(hipStreamSynchronize(st));
        // every later kernel runs again (queued behind the halted iteration)
        mf::launch_set_i32(g->halt_d, 0, st);
    }
    while (!finished) {
        bool queued = false, ended = false;
        int depth = 0;
        mf_status rc = relabel_and_worklist(g, m, &levels, &depth, queue ? &tail : nullptr, &queued);
        if (rc != MF_OK) return rc;
        if (tail_rc != MF_OK) return tail_rc;
        const DevCounters& c = *m.L.ctr_h;
        // the relabel's worklist (after queued rounds, the first round set its sizes aside)
        const int active = queued ? c.wl_in[3] : c.wl[3];  // (set aside by the next-worklist build)
        active_sum += active;
        capped += c.bfs_capped != 0;
        if (active == 0) {
            *value = (int64_t)c.e_t + (int64_t)c.deficit_sum;
            exact = !c.bfs_capped;
            break;
        }
        if (++iters > g->max_iter) {
            if (m.L.main) g->last_iterations = iters;
            return MF_ERR_NOT_CONVERGED;
        }
        int64_t R = std::min<int64_t>(g->round_max, std::max<int64_t>(g->round_min, depth / g->round_div));
        int cnt[3];
        int32_t* cur[3];
        if (g->trace_gr)
            std::fprintf(stderr, "[loop] relabel %lld depth %lld active %d (rows by bin %d %d %d) rounds %lld\n",
                         (long long)iters, (long long)depth, active, c.wl[0], c.wl[1], c.wl[2], (long long)R);
        // several rounds on the main lane: later worklists come from the
        // previous one plus the vertices the round activated, not a scan of
        // every vertex
        const bool incremental = R > 1 && m.L.main && !m.pull && !m.topology && g->incremental_rounds;
        auto thin = [&](const int b[3]) {
            return incremental && g->rn_limit > 0 && b[2] == 0 && b[0] + b[1] <= g->rn_limit;
        };
        LoopMode rm = m;
        if (incremental) {
            rc = ensure_round_lists(g);
            if (rc != MF_OK) return rc;
            rm.dg.act = g->act_list;
            rm.dg.act_cnt = &m.L.ctr->act;
            rm.dg.act_cap = g->n;
        }
        int64_t done = 0;  // rounds run on this relabel
        // the last round left no active vertex (round terms cleared): the
        // value, if every sink is still at height 0 (else the next relabel
        // certifies)
        auto end_after_round = [&]() -> mf_status {
            if (!shortcut) return MF_OK;
            mf::launch_value_if_empty(m.dg, m.L.ctr, -1, st);
            MF_HIP(hipGetLastError());
            mf_status r2 = read_lane(g, m.L);
            if (r2 != MF_OK) return r2;
            if (c.round_raised == 0) {
                *value = (int64_t)c.round_e_t + (int64_t)c.round_deficit;
                ended = true;
            }
            return MF_OK;
        };
        if (queued) {
            // two rounds ran; the second one's worklist and activations are on the device
            done = 2;
            rounds += 2;
            for (int b = 0; b < 3; ++b) {
                cur[b] = g->wlb[b];
                cnt[b] = c.wl[b];
            }
            if (c.wl[3] == 0 && shortcut && c.round_raised == 0) {  // the first round left no active vertex
                *value = (int64_t)c.round_e_t + (int64_t)c.round_deficit;
                break;
            }
            if (thin(cnt)) R = std::max<int64_t>(R, THIN_ROUNDS_MIN);
            if (c.wl[3] == 0 || R <= 2) continue;  // certified by the next relabel
            active_sum += c.wl[3];
        } else {
            for (int b = 0; b < 3; ++b) {
                cur[b] = m.L.wl[b];
                cnt[b] = c.wl[b];
            }
            // k_build_worklist cleared the activation count; the persistent
            // relabel's worklist did not
            if (incremental && g->persistent_grid > 0) mf::launch_zero_act(m.L.ctr, st);
        }
        for (;;) {
            if (done > 0) {
                if (done >= R) break;
                bool rebuilt = false;
                if (incremental) {
                    count_epochs(g, st, 1);
                    int32_t* nxt[3];
                    for (int b = 0; b < 3; ++b) nxt[b] = cur[b] == m.L.wl[b] ? g->wlb[b] : m.L.wl[b];
                    timed(g, m.L, mf::KC_WL, [&] {
                        mf::launch_next_worklist(rm.dg, cur, cnt, nxt[0], nxt[1], nxt[2], g->mark, g->mark + g->n,
                                                 m.L.ctr, st);
                    });
                    MF_HIP(hipGetLastError());
                    rc = read_lane(g, m.L);
                    if (rc != MF_OK) return rc;
                    if (c.act <= g->n) {
                        for (int b = 0; b < 3; ++b) cur[b] = nxt[b];
                        rebuilt = true;
                        mf::launch_zero_act(m.L.ctr, st);
                    }
                    // else activations were dropped: scan every vertex instead
                }
                if (!rebuilt) {
                    mf::launch_zero_loop_counters(m.L.ctr, st);
                    timed(g, m.L, mf::KC_WL, [&] {
                        mf::launch_build_worklist(m.dg, m.L.wl[0], m.L.wl[1], m.L.wl[2], m.L.ctr, m.topology,
                                                  m.sign, st);
                    });
                    MF_HIP(hipGetLastError());
                    rc = read_lane(g, m.L);
                    if (rc != MF_OK) return rc;
                    for (int b = 0; b < 3; ++b) cur[b] = m.L.wl[b];
                }
                if (g->trace_gr)
                    std::fprintf(stderr, "[loop]   round %lld active %d (rows by bin %d %d %d)\n", (long long)done,
                                 c.wl[3], c.wl[0], c.wl[1], c.wl[2]);
                if (c.wl[3] == 0) {
                    if (!rebuilt) mf::launch_round_terms_clear(m.L.ctr, st);  // (the full build's)
                    rc = end_after_round();
                    if (rc != MF_OK) return rc;
                    break;  // else certified by the next relabel
                }
                active_sum += c.wl[3];
                cnt[0] = c.wl[0];
                cnt[1] = c.wl[1];
                cnt[2] = c.wl[2];
            }
            // a short list without workgroup-bin rows: rounds in one workgroup,
            // many per launch, until the list grows or empties
            if (thin(cnt)) R = std::max<int64_t>(R, THIN_ROUNDS_MIN);
            if (thin(cnt) && R - done >= 4) {
                int32_t* other[3];
                for (int b = 0; b < 3; ++b) other[b] = cur[b] == m.L.wl[b] ? g->wlb[b] : m.L.wl[b];
                const int most = (int)std::min<int64_t>(R - done, INT_MAX / 2);
                count_epochs(g, st, most);
                mf::launch_rounds_narrow(rm.dg, cur, other, g->mark, g->mark + g->n, m.L.ctr, kc_for_bin(g, 0), most,
                                         g->rn_limit, st);
                mf::launch_zero_act(m.L.ctr, st);  // the last round's activations are in the new list
                MF_HIP(hipGetLastError());
                rc = read_lane(g, m.L);
                if (rc != MF_OK) return rc;
                if (c.rn_rounds > 0) {
                    if (c.rn_set)
                        for (int b = 0; b < 3; ++b) cur[b] = other[b];
                    done += c.rn_rounds;
                    rounds += c.rn_rounds;
                    if (c.wl[3] == 0) {
                        mf::launch_round_terms_clear(m.L.ctr, st);
                        rc = end_after_round();
                        if (rc != MF_OK) return rc;
                        break;
                    }
                    if (done >= R) break;
                    active_sum += c.wl[3];
                    cnt[0] = c.wl[0];
                    cnt[1] = c.wl[1];
                    cnt[2] = c.wl[2];
                }
            }
            rc = push_round(g, rm, cur, cnt);
            if (rc != MF_OK) return rc;
            ++rounds;
            ++done;
        }
        if (ended) break;
    }
    if (shortcut) g->heights_exact = exact;
    if (m.L.main) {
        g->last_iterations = iters;
        g->last_levels = levels;
        g->last_active_sum = active_sum;
        g->last_rounds = rounds;
        g->last_capped = capped;
    }
    return MF_OK;
}

// One sweep on the heights the previous solve left: worklist, push-relabel,
// remove-invalid-edges.  Only the loop that follows certifies the value.
mf_status warm_sweep(mf_graph* g) {
    hipStream_t st = g->stream;
    LoopMode m = solve_mode(g);
    mf::launch_zero_loop_counters(g->ctr, st);
    timed(g, mf::KC_WL, [&] {
        mf::launch_build_worklist(m.dg, g->wl[0], g->wl[1], g->wl[2], g->ctr, m.topology, 1, st);
    });
    // sized on the device: no read-back between the build and the sweep
    const int bounds[3] = {(int)g->n, (int)g->n, (int)g->n};
    timed(g, mf::KC_PR, [&] {
        mf::launch_push_relabel_round(m.dg, g->wl, bounds, kc_for_bin(g, 0), kc_for_bin(g, 2), false, st, g->ctr->wl);
    });
    timed(g, mf::KC_RIE, [&] { mf::launch_remove_invalid_round(m.dg, g->wl, bounds, g->ctr, st, g->ctr->wl); });
    MF_HIP(hipGetLastError());
    return MF_OK;
}

mf_status check_handle(mf_graph* g) {
    if (!g) return MF_ERR_INVALID;
    if (g->poisoned) return MF_ERR_DEVICE;
    if (g->offloaded) return MF_ERR_STATE;
    g->dg.count_bytes = g->prof_mask != 0;
    if (hipSetDevice(g->device) != hipSuccess) {
        g->poisoned = true;
        return MF_ERR_DEVICE;
    }
    return MF_OK;
}

// Rows ran out of slack: re-lay them on the device with room for need[v]
// more pairs plus fresh slack.  Excess and heights stay.
mf_status relayout(mf_graph* g) {
    hipStream_t st = g->stream;
    mf::RelayoutPlan p{};
    p.V = g->n;
    p.row_ptr = g->dg.row_ptr;
    p.row_len = g->dg.row_len;
    p.row_sorted = g->dg.row_sorted;
    p.need = g->need;
    p.slack_min = g->slack_min;
    p.slack_pct = g->slack_pct;
    // a stream of inserts that outgrew the slack once will again: each
    // relayout doubles the fresh slack (up to 8x), so relayouts get rarer
    // geometrically; slots past a row's length are never scanned
    p.slack_shift = std::min(g->relayouts + 1, 3);
    mf::SlotArrays a{g->dg.cr, g->dg.rev, g->dg.cap, g->dg.capsum};
    int64_t S = 0;
    mf_status rc = mf::relayout_device(p, &a, g->slot_cap, &S, g->dg.row_ptr, g->dg.row_sorted, st, g->mem);
    if (rc != MF_OK) {
        if (rc == MF_ERR_DEVICE) g->poisoned = true;
        return rc;
    }
    g->dg.cr = a.cr;
    g->dg.rev = a.rev;
    g->dg.cap = a.cap;
    g->dg.capsum = a.capsum;
    g->slot_cap = S;
    // arrays whose size follows the slot count
    dfree(g, g->win);
    dfree(g, g->q[0]);
    dfree(g, g->q[1]);
    g->q_cap = (int64_t)g->n + S / mf::GR_CHUNK + 64;
    if (dalloc(g, &g->win, S) != hipSuccess || dalloc(g, &g->q[0], g->q_cap) != hipSuccess ||
        dalloc(g, &g->q[1], g->q_cap) != hipSuccess) {
        g->poisoned = true;
        return MF_ERR_OUT_OF_MEMORY;
    }
    mf::launch_fill_i32(g->win, -1, S, st);
    MF_HIP(hipGetLastError());
    g->relayouts++;
    return MF_OK;
}

mf_status push_pull_phase(mf_graph* g);

// Algorithm 5 after the updates are on the device.
// The batch scratch one repair runs on: the handle's own buffers, or the
// GPU's static array (allocation-free entry point).
struct BatchScratch {
    int32_t* slot_of;
    int32_t* touched;
    mf::BatchTable tb;
};

BatchScratch handle_scratch(mf_graph* g) { return BatchScratch{g->slot_of, g->touched, g->tb}; }

// may_allocate false: rows without room for their inserts end the call with
// MF_ERR_OUT_OF_MEMORY (nothing applied) instead of a relayout.
mf_status apply_batch_dev(mf_graph* g, const mf_update* d_upd, int64_t k, int64_t* value, const BatchScratch& bs,
                          bool may_allocate) {
    hipStream_t st = g->stream;
    g->last_new_pairs = 0;
    for (int attempt = 0; attempt < 3; ++attempt) {
        mf::launch_clear_counters(g->ctr, st);
        // The validation, then everything else queued right behind it, with
        // no host read of its outcome in between: the batch kernels leave at
        // once on a rejected batch (nothing applied; the solve that follows
        // finds the graph as the last call left it, at its max flow), and
        // the host learns the outcome from the counters the solve reads.
        timed(g, mf::KC_BATCH, [&] {
            mf::launch_batch_locate(g->dg, d_upd, k, bs.slot_of, g->win, bs.tb, g->need, g->ctr, st);
            mf::launch_batch_insert(g->dg, bs.tb, g->ctr, g->nslots_d, st);
            mf::launch_batch_apply(g->dg, d_upd, k, bs.slot_of, g->win, bs.tb, bs.touched, g->ctr, st);
            mf::launch_batch_clamp(g->dg, d_upd, k, bs.touched, g->ctr, st);
            mf::launch_batch_cleanup(bs.tb, g->need, bs.slot_of, g->win, k, g->ctr, st);
        });
        timed(g, mf::KC_INIT, [&] { mf::launch_saturate_source(g->dg, g->ctr, st); });
        MF_HIP(hipGetLastError());
        mf_status rc = MF_OK;
        if (g->push_pull) {
            // (the push-pull phase reads the counters: a rejected batch
            // ends the call before it changes anything)
            rc = read_counters(g);
            if (rc != MF_OK) return rc;
            const DevCounters& c0 = *g->ctr_h;
            if (!(c0.err || c0.cap_overflow || c0.overflow)) rc = push_pull_phase(g);
        } else if (!g->opt.cold_start) {
            rc = warm_sweep(g);
        }
        if (rc == MF_OK) rc = run_loop(g, solve_mode(g), value);
        if (rc != MF_OK) {
            // a solve that failed may have read no counters: read them to
            // tell a rejected batch, whose slots and scratch must be put right
            mf_status rc2 = read_counters(g);
            if (rc2 != MF_OK) return rc2;
        }
        const DevCounters c = *g->ctr_h;  // the batch's outcome (the loop kernels leave these words alone)
        if (c.err || c.cap_overflow || c.overflow) {
            rc = MF_OK;
            if (c.overflow && !c.err && !c.cap_overflow) {
                // need[] still holds the per-row demand (the cleanup left the
                // scratch alone): re-lay, then retry
                if (may_allocate) rc = relayout(g);
                else rc = MF_ERR_OUT_OF_MEMORY;
                if (g->poisoned) return MF_ERR_DEVICE;
            }
            mf::launch_batch_cleanup(bs.tb, g->need, bs.slot_of, g->win, k, nullptr, st);
            MF_HIP(hipGetLastError());
            MF_HIP(hipStreamSynchronize(st));
            if (rc != MF_OK) return rc;
            if (c.err) return MF_ERR_INVALID;
            if (c.cap_overflow) return MF_ERR_OVERFLOW;
            continue;
        }
        if (rc != MF_OK) return rc;
        g->last_new_pairs = c.new_pairs;
        g->dg.used_slots += 2 * (int64_t)c.new_pairs;  // (the insert kernel moved the device copy on)
        return MF_OK;
    }
    return MF_ERR_OUT_OF_MEMORY;  // slack could not be made to fit
}

// The pull side's lane: its own stream (default priority), queues sized like
// the main lane's, worklists, bitmaps, counters and heights.
mf_status ensure_lane2(mf_graph* g) {
    const int64_t n = g->n;
    if (!g->stream2 && hipStreamCreateWithFlags(&g->stream2, hipStreamNonBlocking) != hipSuccess)
        return MF_ERR_DEVICE;
    if (!g->ctr2_h && hipHostMalloc((void**)&g->ctr2_h, sizeof(DevCounters), hipHostMallocDefault) != hipSuccess)
        return MF_ERR_OUT_OF_MEMORY;
    if (g->q2_cap < g->q_cap) {
        dfree(g, g->q2[0]);
        dfree(g, g->q2[1]);
        g->q2_cap = 0;
        if (dalloc(g, &g->q2[0], g->q_cap) != hipSuccess || dalloc(g, &g->q2[1], g->q_cap) != hipSuccess)
            return MF_ERR_OUT_OF_MEMORY;
        g->q2_cap = g->q_cap;
    }
    if (!g->h2) {
        g->bits2.nwords = g->bits.nwords;
        if (dalloc(g, &g->wl2[0], n) != hipSuccess || dalloc(g, &g->wl2[1], n) != hipSuccess ||
            dalloc(g, &g->wl2[2], n) != hipSuccess ||
            dalloc(g, &g->bits2.visited, 4 * (int64_t)g->bits2.nwords) != hipSuccess ||
            dalloc(g, &g->ctr2, 1) != hipSuccess || dalloc(g, &g->h2, n) != hipSuccess) {
            free_lane2(g);
            return MF_ERR_OUT_OF_MEMORY;
        }
        g->bits2.fb = g->bits2.visited + g->bits2.nwords;
        mf::launch_clear_counters(g->ctr2, g->stream2);
        MF_HIP(hipStreamSynchronize(g->stream2));
    }
    return ensure_med(g, g->med2);
}

// Section 5.2's O2 after a batch: the source side S of the last terminating
// relabel (h = |V|) and the rest T were separated by a saturated cut; the
// batch may have opened it.  Saturate every residual S -> T slot again, then
// run at the same time, on two streams, push-relabel inside T (excess flows
// to t and T's deficits, relabels seeded only in T) and pull-relabel inside S
// (deficits pull from s and S's excess, forward relabels seeded only in S).
// No residual path leads from S to T, so the two never touch the same vertex
// or slot.  The caller then runs the ordinary loop over the whole graph,
// whose fresh relabel certifies the value.
mf_status push_pull_phase(mf_graph* g) {
    hipStream_t st = g->stream;
    mf_status rc = ensure_lane2(g);
    if (rc != MF_OK) return rc;
    mf::launch_mark_side(g->dg, g->side, st);
    mf::launch_saturate_cut(g->dg, g->side, g->slot_cap, st);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(st));
    LoopMode push_t = solve_mode(g);
    push_t.dg.side = g->side;
    push_t.dg.side_keep = 0;
    LoopMode pull_s = push_t;
    pull_s.dg.side_keep = 1;
    pull_s.dg.h = g->h2;
    pull_s.dg.root = g->s;
    pull_s.dg.pinned = g->t;
    pull_s.seed_deficits = -1;  // overflowing vertices of S are bases of the pull heights
    pull_s.forward = true;
    pull_s.sign = -1;
    pull_s.pull = true;
    pull_s.rie = false;
    Lane& L2 = pull_s.L;
    L2.stream = g->stream2;
    L2.q[0] = g->q2[0];
    L2.q[1] = g->q2[1];
    for (int b = 0; b < 3; ++b) L2.wl[b] = g->wl2[b];
    L2.bits = g->bits2;
    L2.ctr = g->ctr2;
    L2.ctr_h = g->ctr2_h;
    set_med(L2, g->med2);
    L2.main = false;
    int64_t v1 = 0, v2 = 0;
    mf_status rc2 = MF_OK;
    if (g->persistent_grid > 0) {
        // two cooperative launches must not wait on each other: one side after the other
        mf::launch_zero_loop_counters(g->ctr, st);
        rc = run_loop(g, push_t, &v1);
        if (rc != MF_OK) return rc;
        mf::launch_zero_loop_counters(g->ctr2, g->stream2);
        return run_loop(g, pull_s, &v2);
    }
    std::thread pull_thread;
    try {
        pull_thread = std::thread([&] {
            if (hipSetDevice(g->device) != hipSuccess) {
                rc2 = MF_ERR_DEVICE;
                return;
            }
            mf::launch_zero_loop_counters(g->ctr2, g->stream2);
            rc2 = run_loop(g, pull_s, &v2);
        });
    } catch (...) {
        return MF_ERR_OUT_OF_MEMORY;  // no thread: nothing was launched
    }
    mf::launch_zero_loop_counters(g->ctr, st);
    rc = run_loop(g, push_t, &v1);
    pull_thread.join();
    if (rc != MF_OK) return rc;
    if (rc2 != MF_OK) {
        if (rc2 == MF_ERR_DEVICE) g->poisoned = true;
        return rc2;
    }
    return MF_OK;
}

// Whether everything prepare_loop takes is there (the allocation-free repair
// runs only then).
bool loop_ready(const mf_graph* g) {
    return g->act_list && g->mark && g->wlb[0] && g->snap_h[0] && g->snap_h[1] && g->snap_ev[0] && g->snap_ev[1] &&
           (!g->push_pull || (g->h2 && g->q2_cap >= g->q_cap)) && (!g->bfs_cap || g->dg.h_prev);
}

// Everything a solve or repair may allocate, taken before it changes any
// state: a failed allocation then leaves the graph as it was.
mf_status prepare_loop(mf_graph* g) {
    mf_status rc = ensure_round_lists(g);
    if (rc == MF_OK) rc = ensure_snapshots(g);
    if (rc == MF_OK && g->push_pull) rc = ensure_lane2(g);
    if (rc == MF_OK && g->bfs_cap && !g->dg.h_prev && dalloc(g, &g->dg.h_prev, g->n) != hipSuccess)
        rc = MF_ERR_OUT_OF_MEMORY;
    if (rc == MF_OK) rc = ensure_med(g, g->med);
    return rc;
}

struct CallTimer {
    mf_graph* g;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    explicit CallTimer(mf_graph* gg) : g(gg) {}
    ~CallTimer() {
        g->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

}  // namespace

extern "C" {

void mf_default_options(mf_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(mf_options);
    opt->device = -1;
}

const char* mf_status_string(mf_status status) {
    switch (status) {
        case MF_OK: return "ok";
        case MF_ERR_INVALID: return "invalid argument";
        case MF_ERR_OUT_OF_MEMORY: return "out of memory";
        case MF_ERR_OVERFLOW: return "capacity overflow";
        case MF_ERR_DEVICE: return "device error";
        case MF_ERR_NOT_CONVERGED: return "iteration cap reached";
        case MF_ERR_STATE: return "call order";
    }
    return "unknown status";
}

mf_status mf_graph_load(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* cap, int32_t s, int32_t t, const mf_options* opt,
                        mf_graph** out) {
    if (!out) return MF_ERR_INVALID;
    *out = nullptr;
    mf_options o;
    mf_default_options(&o);
    if (opt) {
        if (opt->struct_size != sizeof(mf_options)) return MF_ERR_INVALID;
        o = *opt;
    }
    int32_t slack_min = o.insert_slack_min > 0 ? o.insert_slack_min : 8;
    int32_t slack_pct = o.insert_slack_pct > 0 ? o.insert_slack_pct : 12;
    mf::Tuning tuning;
    if (mf::resolve_tuning(o, &tuning) != MF_OK) return MF_ERR_INVALID;
    if ((o.alloc == nullptr) != (o.free == nullptr)) return MF_ERR_INVALID;
    mf::HostBiCSR b;
    mf_status rc = mf::build_bicsr(n, m, src, dst, cap, s, t, slack_min, slack_pct, &b);
    if (rc != MF_OK) return rc;

    mf_graph* g = new (std::nothrow) mf_graph();
    if (!g) return MF_ERR_OUT_OF_MEMORY;
    g->mem.alloc_fn = o.alloc;
    g->mem.free_fn = o.free;
    g->mem.ctx = o.alloc_ctx;
    g->opt = o;
    g->n = n;
    g->s = s;
    g->t = t;
    g->slack_min = slack_min;
    g->slack_pct = slack_pct;
    g->pairs = b.pairs;
    g->m_unique = b.m_unique;
    apply_tuning(g, tuning);
    g->push_pull = o.push_pull != 0;
    g->max_iter = o.max_iterations > 0 ? o.max_iterations : 4 * (int64_t)n + 1000;
    auto fail = [&](mf_status r) {
        free_all(g);
        if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
        delete g;
        return r;
    };
    int dev = o.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(MF_ERR_DEVICE);
    if (hipSetDevice(dev) != hipSuccess) return fail(MF_ERR_DEVICE);
    g->device = dev;
    if (o.stream) {
        g->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) return fail(MF_ERR_DEVICE);
        g->own_stream = true;
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (dalloc(g, &g->dg.bytes_part, (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS) != hipSuccess)
        return fail(MF_ERR_OUT_OF_MEMORY);
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->dg.bytes_part), 0,
                        2 * (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS, g->stream);
    // BFS bitmaps: visited plus a ring of three frontier bitmaps
    g->bits.nwords = (n + 31) / 32;
    if (dalloc(g, &g->bits.visited, 4 * (int64_t)g->bits.nwords) != hipSuccess) return fail(MF_ERR_OUT_OF_MEMORY);
    g->bits.fb = g->bits.visited + g->bits.nwords;
    {
        int coop = 0;
        g->coop_ok = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop;
    }
    g->cus = cus;
    apply_loop_options(g, o);
    g->dg.n = n;
    g->dg.s = s;
    g->dg.t = t;
    g->dg.root = t;
    g->dg.pinned = s;
    g->dg.used_slots = b.pairs;
    if (dalloc(g, &g->nslots_d, 2) != hipSuccess) return fail(MF_ERR_OUT_OF_MEMORY);
    g->dg.nslots = g->nslots_d;
    g->halt_d = reinterpret_cast<int32_t*>(g->nslots_d + 1);
    g->dg.halt = g->halt_d;
    mf::launch_set_i64(g->nslots_d, g->dg.used_slots, g->stream);
    mf::launch_set_i32(g->halt_d, 0, g->stream);
    if (dalloc(g, &g->dg.e, n) != hipSuccess || dalloc(g, &g->dg.h, n) != hipSuccess ||
        dalloc(g, &g->wl[0], n) != hipSuccess || dalloc(g, &g->wl[1], n) != hipSuccess ||
        dalloc(g, &g->wl[2], n) != hipSuccess || dalloc(g, &g->ctr, 1) != hipSuccess ||
        dalloc(g, &g->need, n) != hipSuccess || dalloc(g, &g->side, n) != hipSuccess ||
        dalloc(g, &g->cut_acc, 8) != hipSuccess)
        return fail(MF_ERR_OUT_OF_MEMORY);
    if (hipHostMalloc((void**)&g->ctr_h, sizeof(DevCounters), hipHostMallocDefault) != hipSuccess)
        return fail(MF_ERR_OUT_OF_MEMORY);
    rc = upload_structure(g, b, {});
    if (rc != MF_OK) return fail(rc);
    rc = ensure_med(g, g->med);  // (needs q_cap)
    if (rc != MF_OK) return fail(rc);
    mf::launch_fill_i32(g->need, 0, n, g->stream);
    mf::launch_fill_i32(g->dg.h, 0, n, g->stream);
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->dg.e), 0, 2 * (int64_t)n, g->stream);
    mf::launch_clear_counters(g->ctr, g->stream);
    if (g->medium_blocks > 0) {
        // the process's first cooperative launch carries a one-time setup of
        // several ms: pay it here rather than in the first solve (limit -1:
        // the kernel leaves at its first frontier check, changing nothing but
        // the level counter, which every relabel resets)
        const mf::MedQueue mq{g->med.q, g->med.rec, g->med.seg};
        if (mf::launch_gr_medium(g->dg, 0, g->q[0], g->q[1], g->ctr, g->bits, g->tune, -1, false,
                                 std::min(g->medium_blocks, g->med.blocks), mq, g->stream) != hipSuccess) {
            (void)hipGetLastError();
            g->coop_broken = true;
        }
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(g->stream) != hipSuccess)
        return fail(MF_ERR_DEVICE);
    *out = g;
    return MF_OK;
}

mf_status mf_maxflow(mf_graph* g, int64_t* value) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!value) return MF_ERR_INVALID;
    CallTimer timer(g);
    hipStream_t st = g->stream;
    rc = prepare_loop(g);
    if (rc != MF_OK) return rc;
    g->solved = false;
    mf::launch_clear_counters(g->ctr, st);
    timed(g, mf::KC_INIT, [&] {
        mf::launch_reset(g->dg, g->slot_cap, st);
        mf::launch_saturate_source(g->dg, g->ctr, st);
        if (g->push_pull) mf::launch_saturate_sink(g->dg, st);  // static push-pull (Section 5.2)
    });
    MF_HIP(hipGetLastError());
    int64_t v = 0;
    rc = run_loop(g, solve_mode(g), &v);
    settle_events(g);
    fold_bytes(g);
    if (rc != MF_OK) return rc;
    g->solved = true;
    g->last_value = v;
    *value = v;
    return MF_OK;
}

// After a repair: errors found before anything changed (invalid updates,
// capacity overflow, rows the slack could not be made to fit) leave the last
// solve standing.
static mf_status finish_apply(mf_graph* g, mf_status rc, int64_t v, int64_t* value) {
    if (rc == MF_ERR_INVALID || rc == MF_ERR_OVERFLOW || rc == MF_ERR_OUT_OF_MEMORY) {
        g->solved = true;  // nothing was applied
        return rc;
    }
    if (rc != MF_OK) return rc;
    g->solved = true;
    g->last_value = v;
    *value = v;
    return MF_OK;
}

static mf_status apply_common(mf_graph* g, const mf_update* upd, int64_t k, int64_t* value, bool on_device) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!value || k < 0 || (k > 0 && !upd)) return MF_ERR_INVALID;
    if (!g->solved) return MF_ERR_STATE;
    if (k > INT_MAX / 2) return MF_ERR_INVALID;
    CallTimer timer(g);
    if (k == 0) {
        *value = g->last_value;
        return MF_OK;
    }
    rc = ensure_batch_capacity(g, k);
    if (rc == MF_OK) rc = prepare_loop(g);
    if (rc != MF_OK) return rc;
    const mf_update* d_upd = upd;
    if (!on_device) {
        // through pinned staging, so that the copy is a plain asynchronous DMA
        // queued behind the work still on the stream (the last call's copy out
        // of the staging buffer finished before that call returned)
        std::memcpy(g->upd_h, upd, sizeof(mf_update) * (size_t)k);
        if (g->upd_h_dev) {
            // a copy kernel reads the pinned buffer over the bus (no DMA-engine round trip)
            mf::launch_copy_i32(reinterpret_cast<int32_t*>(g->upd), reinterpret_cast<const int32_t*>(g->upd_h_dev),
                                3 * k, g->stream);
            MF_HIP(hipGetLastError());
        } else {
            MF_HIP(hipMemcpyAsync(g->upd, g->upd_h, sizeof(mf_update) * (size_t)k, hipMemcpyHostToDevice,
                                  g->stream));
        }
        d_upd = g->upd;
    }
    g->solved = false;
    int64_t v = 0;
    rc = apply_batch_dev(g, d_upd, k, &v, handle_scratch(g), true);
    settle_events(g);
    fold_bytes(g);
    return finish_apply(g, rc, v, value);
}

mf_status mf_apply_batch(mf_graph* g, const mf_update* upd, int64_t k, int64_t* value) {
    return apply_common(g, upd, k, value, false);
}

mf_status mf_apply_batch_device(mf_graph* g, const mf_update* d_upd, int64_t k, int64_t* value) {
    return apply_common(g, d_upd, k, value, true);
}

mf_status mf_apply_batch_device_noalloc(mf_graph* g, const mf_update* d_upd, int64_t k, int64_t* value) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!value || k < 0 || (k > 0 && !d_upd) || k > mf::NOALLOC_MAX_UPDATES) return MF_ERR_INVALID;
    if (!g->solved || !loop_ready(g)) return MF_ERR_STATE;
    CallTimer timer(g);
    if (k == 0) {
        *value = g->last_value;
        return MF_OK;
    }
    mf::NoallocScratch ns;
    rc = mf::noalloc_scratch(g->device, &ns);
    if (rc != MF_OK) return rc;
    int32_t tcap = 64;
    while (tcap < 2 * k) tcap *= 2;
    const BatchScratch bs{ns.slot_of, ns.touched, mf::BatchTable{ns.table_key, ns.table_win, ns.table_slot, tcap}};
    // the array keeps the last call's contents: the part of the table this
    // batch uses starts empty (slot_of and touched are written before read)
    hipStream_t st = g->stream;
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(bs.tb.key), -1, 2 * (int64_t)tcap, st);
    mf::launch_fill_i32(bs.tb.win, -1, 2 * (int64_t)tcap, st);
    MF_HIP(hipGetLastError());
    g->solved = false;
    g->no_capture = true;
    int64_t v = 0;
    rc = apply_batch_dev(g, d_upd, k, &v, bs, false);
    g->no_capture = false;
    settle_events(g);
    fold_bytes(g);
    return finish_apply(g, rc, v, value);
}

mf_status mf_min_cut(mf_graph* g, uint8_t* source_side, int64_t* cut_capacity) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!cut_capacity) return MF_ERR_INVALID;
    if (!g->solved) return MF_ERR_STATE;
    hipStream_t st = g->stream;
    if (!g->heights_exact) {
        // the solve ended after a round (valid heights, not distances): the
        // cut of Sections 3.1 / 4.3 is read from a fresh relabel of the same
        // residual graph, which the solve would have ended with
        int64_t levels = 0;
        int depth = 0;
        LoopMode m = solve_mode(g);
        m.topology = false;
        rc = global_relabel(g, m, &levels, &depth);
        if (rc != MF_OK) return rc;
        g->heights_exact = true;
    }
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->cut_acc), 0, 2, st);
    mf::launch_cut(g->dg, g->side, g->cut_acc, st);
    MF_HIP(hipGetLastError());
    unsigned long long c = 0;
    MF_HIP(hipMemcpyAsync(&c, g->cut_acc, sizeof(c), hipMemcpyDeviceToHost, st));
    if (source_side) MF_HIP(hipMemcpyAsync(source_side, g->side, (size_t)g->n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    *cut_capacity = (int64_t)c;
    return MF_OK;
}

mf_status mf_get_flow(mf_graph* g, int64_t* count, int32_t* src, int32_t* dst, int32_t* flow) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!count) return MF_ERR_INVALID;
    bool want = src && dst && flow;
    if ((src || dst || flow) && !want) return MF_ERR_INVALID;
    if (!g->solved) return MF_ERR_STATE;
    hipStream_t st = g->stream;
    unsigned long long cnt = 0;
    if (!want) {
        mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->cut_acc), 0, 2, st);
        mf::launch_flow_slots(g->dg, nullptr, g->cut_acc, st);
        MF_HIP(hipGetLastError());
        MF_HIP(hipMemcpyAsync(&cnt, g->cut_acc, sizeof(cnt), hipMemcpyDeviceToHost, st));
        MF_HIP(hipStreamSynchronize(st));
        *count = (int64_t)cnt;
        return MF_OK;
    }
    const int32_t n = g->n;
    const int64_t S = g->slot_cap;
    int2* cr2 = nullptr;
    int64_t* e2 = nullptr;
    int32_t* h2 = nullptr;
    int32_t* fslot = nullptr;
    auto release = [&] {
        dfree(g, cr2);
        dfree(g, e2);
        dfree(g, h2);
        dfree(g, fslot);
    };
    // every exit, the early error returns of MF_HIP included, releases the copies
    struct Guard {
        std::function<void()> f;
        ~Guard() { f(); }
    } guard{release};
    if (dalloc(g, &cr2, S) != hipSuccess || dalloc(g, &e2, n) != hipSuccess ||
        dalloc(g, &h2, n) != hipSuccess || dalloc(g, &fslot, S) != hipSuccess) {
        release();
        return MF_ERR_OUT_OF_MEMORY;
    }
    // work on a copy: the retained preflow stays as it is
    MF_HIP(hipMemcpyAsync(cr2, g->dg.cr, sizeof(int2) * S, hipMemcpyDeviceToDevice, st));
    MF_HIP(hipMemcpyAsync(e2, g->dg.e, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st));
    LoopMode to_source = solve_mode(g);  // the handle's lane; the graph arrays are the copies
    to_source.topology = false;
    to_source.dg.cr = cr2;
    to_source.dg.e = e2;
    to_source.dg.h = h2;
    to_source.dg.root = g->s;
    to_source.dg.pinned = g->t;
    to_source.seed_deficits = 0;
    to_source.rie = false;
    LoopMode from_sink = to_source;
    from_sink.dg.root = g->t;
    from_sink.dg.pinned = g->s;
    from_sink.forward = true;
    from_sink.sign = -1;
    from_sink.pull = true;
    int64_t dummy = 0;
    int64_t it_keep = g->last_iterations, lv_keep = g->last_levels, act_keep = g->last_active_sum;
    rc = run_loop(g, to_source, &dummy);
    if (rc == MF_OK) rc = run_loop(g, from_sink, &dummy);
    g->last_iterations = it_keep;
    g->last_levels = lv_keep;
    g->last_active_sum = act_keep;
    if (rc != MF_OK) {
        release();
        return rc;
    }
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->cut_acc), 0, 2, st);
    mf::launch_flow_slots(to_source.dg, fslot, g->cut_acc, st);
    MF_HIP(hipGetLastError());
    std::vector<int32_t> fs((size_t)S), rp((size_t)n + 1), rl((size_t)n);
    std::vector<int2> cr((size_t)S);
    MF_HIP(hipMemcpyAsync(&cnt, g->cut_acc, sizeof(cnt), hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(fs.data(), fslot, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(cr.data(), g->dg.cr, sizeof(int2) * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(rp.data(), g->dg.row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(rl.data(), g->dg.row_len, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    release();
    if ((int64_t)cnt > *count) return MF_ERR_INVALID;  // caller's arrays are too short
    // emit rows in order, each row's entries by column
    int64_t k = 0;
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int32_t u = 0; u < n; ++u) {
        row.clear();
        for (int32_t q = 0; q < rl[(size_t)u]; ++q) {
            int32_t j = rp[(size_t)u] + q;
            if (fs[(size_t)j] >= 0) row.push_back({cr[(size_t)j].x, fs[(size_t)j]});
        }
        std::sort(row.begin(), row.end());
        for (auto& p : row) {
            src[k] = u;
            dst[k] = p.first;
            flow[k] = p.second;
            ++k;
        }
    }
    *count = k;
    return MF_OK;
}

mf_status mf_get_edges(mf_graph* g, int64_t* count, int32_t* src, int32_t* dst, int32_t* cap) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!count) return MF_ERR_INVALID;
    bool want = src && dst && cap;
    if ((src || dst || cap) && !want) return MF_ERR_INVALID;
    hipStream_t st = g->stream;
    const int32_t n = g->n;
    const int64_t S = g->slot_cap;
    std::vector<int32_t> cp((size_t)S), rp((size_t)n + 1), rl((size_t)n);
    std::vector<int2> cr((size_t)S);
    MF_HIP(hipMemcpyAsync(cp.data(), g->dg.cap, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(cr.data(), g->dg.cr, sizeof(int2) * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(rp.data(), g->dg.row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(rl.data(), g->dg.row_len, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    int64_t total = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t q = 0; q < rl[(size_t)u]; ++q) total += cp[(size_t)(rp[(size_t)u] + q)] > 0;
    if (!want) {
        *count = total;
        return MF_OK;
    }
    if (total > *count) return MF_ERR_INVALID;
    int64_t k = 0;
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int32_t u = 0; u < n; ++u) {
        row.clear();
        for (int32_t q = 0; q < rl[(size_t)u]; ++q) {
            int32_t j = rp[(size_t)u] + q;
            if (cp[(size_t)j] > 0) row.push_back({cr[(size_t)j].x, cp[(size_t)j]});
        }
        std::sort(row.begin(), row.end());
        for (auto& p : row) {
            src[k] = u;
            dst[k] = p.first;
            cap[k] = p.second;
            ++k;
        }
    }
    *count = k;
    return MF_OK;
}

mf_status mf_graph_offload(mf_graph* g) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    hipStream_t st = g->stream;
    const int64_t S = g->slot_cap, n = g->n;
    mf_graph::HostCopy& c = g->hc;
    if (c.slots < S) {
        free_host_copy(g);
        if (halloc(&c.cr, S) || halloc(&c.rev, S) || halloc(&c.cap, S) || halloc(&c.capsum, S) ||
            halloc(&c.row_ptr, n + 1) || halloc(&c.row_len, n) || halloc(&c.row_sorted, n) || halloc(&c.h, n) ||
            halloc(&c.e, n)) {
            free_host_copy(g);
            return MF_ERR_OUT_OF_MEMORY;
        }
        c.slots = S;
    }
    MF_HIP(hipMemcpyAsync(c.cr, g->dg.cr, sizeof(int2) * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.rev, g->dg.rev, 4 * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.cap, g->dg.cap, 4 * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.capsum, g->dg.capsum, 4 * S, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.row_ptr, g->dg.row_ptr, 4 * (n + 1), hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.row_len, g->dg.row_len, 4 * n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.row_sorted, g->dg.row_sorted, 4 * n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.h, g->dg.h, 4 * n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipMemcpyAsync(c.e, g->dg.e, 8 * n, hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    free_device_state(g);
    g->offloaded = true;
    return MF_OK;
}

mf_status mf_graph_restore(mf_graph* g) {
    if (!g) return MF_ERR_INVALID;
    if (g->poisoned) return MF_ERR_DEVICE;
    if (!g->offloaded) return MF_ERR_STATE;
    if (hipSetDevice(g->device) != hipSuccess) return MF_ERR_DEVICE;
    hipStream_t st = g->stream;
    const int64_t S = g->slot_cap, n = g->n;
    const mf_graph::HostCopy& c = g->hc;
    g->q_cap = n + S / mf::GR_CHUNK + 64;
    if (dalloc(g, &g->dg.row_ptr, n + 1) || dalloc(g, &g->dg.row_len, n) || dalloc(g, &g->dg.row_sorted, n) ||
        dalloc(g, &g->dg.cr, S) || dalloc(g, &g->dg.rev, S) || dalloc(g, &g->dg.cap, S) ||
        dalloc(g, &g->dg.capsum, S) || dalloc(g, &g->win, S) || dalloc(g, &g->q[0], g->q_cap) ||
        dalloc(g, &g->q[1], g->q_cap) || dalloc(g, &g->dg.e, n) || dalloc(g, &g->dg.h, n) ||
        dalloc(g, &g->wl[0], n) || dalloc(g, &g->wl[1], n) || dalloc(g, &g->wl[2], n) || dalloc(g, &g->need, n) ||
        dalloc(g, &g->side, n) || dalloc(g, &g->cut_acc, 8) ||
        dalloc(g, &g->bits.visited, 4 * (int64_t)g->bits.nwords) ||
        dalloc(g, &g->dg.bytes_part, (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS)) {
        free_device_state(g);
        return MF_ERR_OUT_OF_MEMORY;  // still offloaded, state intact on the host
    }
    g->bits.fb = g->bits.visited + g->bits.nwords;
    MF_HIP(hipMemcpyAsync(g->dg.cr, c.cr, sizeof(int2) * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.rev, c.rev, 4 * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.cap, c.cap, 4 * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.capsum, c.capsum, 4 * S, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.row_ptr, c.row_ptr, 4 * (n + 1), hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.row_len, c.row_len, 4 * n, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.row_sorted, c.row_sorted, 4 * n, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.h, c.h, 4 * n, hipMemcpyHostToDevice, st));
    MF_HIP(hipMemcpyAsync(g->dg.e, c.e, 8 * n, hipMemcpyHostToDevice, st));
    mf::launch_fill_i32(g->win, -1, S, st);
    mf::launch_fill_i32(g->need, 0, n, st);
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(g->dg.bytes_part), 0,
                        2 * (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS, st);
    mf::launch_clear_counters(g->ctr, st);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(st));
    g->offloaded = false;
    // the loop's buffers too, so that a repair right after (the allocation-
    // free one included) finds them; if they cannot be had now, the next
    // allocating call takes them
    if (g->solved) (void)prepare_loop(g);
    return MF_OK;
}

mf_status mf_graph_tune(mf_graph* g, const mf_options* opt) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!opt || opt->struct_size != sizeof(mf_options)) return MF_ERR_INVALID;
    mf::Tuning t;
    if (mf::resolve_tuning(*opt, &t) != MF_OK) return MF_ERR_INVALID;
    apply_tuning(g, t);
    apply_loop_options(g, *opt);
    g->max_iter = opt->max_iterations > 0 ? opt->max_iterations : 4 * (int64_t)g->n + 1000;
    return MF_OK;
}

mf_status mf_get_stats(const mf_graph* g, mf_stats* out) {
    if (!g || !out) return MF_ERR_INVALID;
    std::memset(out, 0, sizeof(*out));
    out->n = g->n;
    out->pairs = g->dg.used_slots;
    out->slot_capacity = g->slot_cap;
    out->slots = g->dg.used_slots;
    // slot arrays (col+res, rev, cap, capsum, win), two frontier queues, per-vertex arrays
    out->device_bytes = g->offloaded ? (int64_t)sizeof(DevCounters)
                                     : g->slot_cap * 24 + 2 * g->q_cap * 8 +
                                           (int64_t)g->n * (4 * 3 + 8 + 4 + 12 + 4 + 1) +
                                           g->k_cap * (4 + 4 + 12) + (int64_t)g->tb.capacity * (8 + 8 + 8);
    out->kernel_cycles = g->kc;
    out->relayouts = g->relayouts;
    out->last_iterations = g->last_iterations;
    out->last_bfs_levels = g->last_levels;
    out->last_active_sum = g->last_active_sum;
    out->last_new_pairs = g->last_new_pairs;
    out->last_rounds = g->last_rounds;
    out->last_capped_relabels = g->last_capped;
    out->last_ms = g->last_ms;
    for (int c = 0; c < 8; ++c) {
        out->kernel_ms[c] = g->kernel_ms[c];
        out->kernel_launches[c] = g->kernel_launches[c];
        out->kernel_bytes[c] = g->kernel_bytes[c];
    }
    return MF_OK;
}

mf_status mf_profile(mf_graph* g, int32_t class_mask) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    g->prof_mask = (uint32_t)class_mask & 0xFFu;
    for (int c = 0; c < 8; ++c) {
        g->kernel_ms[c] = 0;
        g->kernel_launches[c] = 0;
        g->kernel_bytes[c] = 0;
    }
    return MF_OK;
}

mf_status mf_debug_initial_labels(mf_graph* g, int32_t* heights, int64_t* excess, int32_t* active,
                                  int32_t* n_active) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    hipStream_t st = g->stream;
    g->solved = false;
    mf::launch_clear_counters(g->ctr, st);
    mf::launch_reset(g->dg, g->slot_cap, st);
    mf::launch_saturate_source(g->dg, g->ctr, st);
    MF_HIP(hipGetLastError());
    int64_t levels = 0;
    int depth = 0;
    LoopMode m = solve_mode(g);
    m.topology = false;
    rc = relabel_and_worklist(g, m, &levels, &depth);
    if (rc != MF_OK) return rc;
    settle_events(g);
    const DevCounters c = *g->ctr_h;
    if (heights) MF_HIP(hipMemcpyAsync(heights, g->dg.h, sizeof(int32_t) * g->n, hipMemcpyDeviceToHost, st));
    if (excess) MF_HIP(hipMemcpyAsync(excess, g->dg.e, sizeof(int64_t) * g->n, hipMemcpyDeviceToHost, st));
    if (active) {
        int off = 0;
        for (int b = 0; b < 3; ++b) {
            if (c.wl[b]) MF_HIP(hipMemcpyAsync(active + off, g->wl[b], sizeof(int32_t) * c.wl[b], hipMemcpyDeviceToHost, st));
            off += c.wl[b];
        }
    }
    MF_HIP(hipStreamSynchronize(st));
    if (n_active) *n_active = c.wl[0] + c.wl[1] + c.wl[2];
    g->last_levels = levels;
    return MF_OK;
}

mf_status mf_debug_round(mf_graph* g, int32_t parts) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (parts < 0 || parts > 3) return MF_ERR_INVALID;
    hipStream_t st = g->stream;
    const LoopMode m = solve_mode(g);
    mf::launch_zero_loop_counters(g->ctr, st);
    mf::launch_build_worklist(m.dg, g->wl[0], g->wl[1], g->wl[2], g->ctr, false, 1, st);
    const int bounds[3] = {(int)g->n, (int)g->n, (int)g->n};
    if (parts & 1)
        mf::launch_push_relabel_round(m.dg, g->wl, bounds, kc_for_bin(g, 0), kc_for_bin(g, 2), false, st,
                                      g->ctr->wl);
    if (parts & 2) mf::launch_remove_invalid_round(m.dg, g->wl, bounds, g->ctr, st, g->ctr->wl);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(st));
    // the heights are no longer those of a terminating relabel
    g->solved = false;
    return MF_OK;
}

mf_status mf_debug_check_invariants(mf_graph* g, int64_t* counts) {
    mf_status rc = check_handle(g);
    if (rc != MF_OK) return rc;
    if (!counts) return MF_ERR_INVALID;
    hipStream_t st = g->stream;
    mf::launch_check_invariants(g->dg, g->cut_acc, st);
    MF_HIP(hipGetLastError());
    MF_HIP(hipMemcpyAsync(counts, g->cut_acc, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    return MF_OK;
}

mf_status mf_debug_atomic_probe(int32_t device, int64_t n, int32_t width, double* ops_per_s) {
    if (!ops_per_s || n < 1 || n > INT_MAX || (width != 4 && width != 8)) return MF_ERR_INVALID;
    if (device >= 0 && hipSetDevice(device) != hipSuccess) return MF_ERR_DEVICE;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return MF_ERR_DEVICE;
    double r = mf::atomic_probe(n, width, st);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (r < 0) return MF_ERR_DEVICE;
    *ops_per_s = r;
    return MF_OK;
}

mf_status mf_debug_selftest(int32_t device) {
    if (device >= 0 && hipSetDevice(device) != hipSuccess) return MF_ERR_DEVICE;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return MF_ERR_DEVICE;
    int fails = mf::device_selftest(st);
    (void)hipStreamDestroy(st);
    return fails == 0 ? MF_OK : MF_ERR_DEVICE;
}

void mf_graph_free(mf_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    free_all(g);
    free_host_copy(g);
    if (g->stream2) (void)hipStreamDestroy(g->stream2);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

}  // extern "C"
