// Batched solve of many independent graphs (C ABI part).
//
// All graphs share pooled device arrays; each graph keeps its own rows,
// residuals, excesses, heights, queues, worklists, bitmaps and counters.  One
// launch solves every graph (one workgroup per graph running the whole loop
// of Algorithm 1 on the device), one more pair of launches repairs every
// graph after its batch of updates (Algorithm 5), so the host synchronises a
// constant number of times per call however many graphs there are.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "mf.h"
#include "mf_internal.h"

using mf::DevCounters;
using mf::GraphSlot;
using mf::GraphUpdates;

struct mf_batch {
    int device = 0;
    mf::DeviceAllocator mem;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t G = 0;
    mf_options opt{};
    mf::GrTune tune{mf::GR_BU_ALPHA, mf::GR_BU_BETA, mf::GR_STAGE_MIN, 0, 0, 0};
    std::vector<int32_t> n, kc;
    int32_t long_cycles = 1;      // push/relabel cycles of the rows a graph's workgroup takes whole
    std::vector<int64_t> vbase, rpbase, sbase, slots, bbase, qbase, used;
    std::vector<int32_t> s_h, t_h;
    int32_t slack_min = 2, slack_pct = 12;
    int32_t relayouts = 0;
    int32_t round_div = 4;
    int32_t bin0 = mf::BIN0_MAX, bin1 = mf::BIN1_MAX;
    int32_t block = 512;                 // threads per graph
    int32_t kc_option = 0;               // 0: round(m/n) per graph
    std::vector<int64_t> m_unique;
    int64_t total_v = 0, total_rp = 0, total_s = 0, total_b = 0, total_q = 0;
    // pools
    int32_t *row_ptr = nullptr, *row_len = nullptr, *row_sorted = nullptr;
    int2* cr = nullptr;
    int32_t *rev = nullptr, *cap = nullptr, *capsum = nullptr, *win = nullptr, *need = nullptr;
    int64_t* e = nullptr;
    int32_t* h = nullptr;
    unsigned* bits = nullptr;
    int2* q = nullptr;
    int32_t* wl = nullptr;
    DevCounters* ctr = nullptr;
    unsigned long long* bytes_part = nullptr;
    GraphSlot* slots_d = nullptr;
    int32_t* order_d = nullptr;
    std::vector<GraphSlot> slots_h;
    // update scratch, grown on demand
    GraphUpdates* gu_d = nullptr;
    mf_update* upd_d = nullptr;
    int32_t *slot_of = nullptr, *touched = nullptr;
    unsigned long long* tkey = nullptr;
    int32_t *twin = nullptr, *tslot = nullptr;
    int64_t upd_cap = 0, tab_cap = 0;
    // relayout scratch, made on first use
    int32_t *gid_d = nullptr, *need_copy = nullptr;
    int64_t* vbase_d = nullptr;
    uint8_t* grow_d = nullptr;
    std::vector<DevCounters> ctr_h;
    bool solved = false, poisoned = false;
    double last_ms = 0;
    // profiling (mf_batch_profile): the solve launch of each call timed with
    // events and its algorithmic bytes counted on the device
    bool prof = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    double kernel_ms = 0, kernel_bytes = 0;
    std::vector<unsigned long long> bytes_h;
};

namespace {

// The batch being built or freed: its allocator serves every pool.
thread_local const mf::DeviceAllocator* t_mem = nullptr;

struct UseAllocator {
    const mf::DeviceAllocator* prev;
    explicit UseAllocator(const mf::DeviceAllocator& m) : prev(t_mem) { t_mem = &m; }
    ~UseAllocator() { t_mem = prev; }
};

template <class T>
hipError_t balloc(T** p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    if (t_mem) return t_mem->allocate((void**)p, bytes);
    return hipMalloc((void**)p, bytes);
}

template <class T>
void bfree(T*& p) {
    if (t_mem) t_mem->release((void*)p);
    else if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void free_batch(mf_batch* b) {
    bfree(b->row_ptr); bfree(b->row_len); bfree(b->row_sorted); bfree(b->cr); bfree(b->rev);
    bfree(b->cap); bfree(b->capsum); bfree(b->win); bfree(b->need); bfree(b->e); bfree(b->h);
    bfree(b->bits); bfree(b->q); bfree(b->wl); bfree(b->ctr); bfree(b->bytes_part);
    bfree(b->slots_d); bfree(b->order_d); bfree(b->gu_d); bfree(b->upd_d); bfree(b->slot_of);
    bfree(b->touched); bfree(b->tkey); bfree(b->twin); bfree(b->tslot);
    bfree(b->gid_d); bfree(b->need_copy); bfree(b->vbase_d); bfree(b->grow_d);
}

#define MFB_HIP(call)              \
    do {                           \
        if ((call) != hipSuccess) { \
            b->poisoned = true;    \
            return MF_ERR_DEVICE;  \
        }                          \
    } while (0)

mf_status read_results(mf_batch* b, int64_t* values) {
    MFB_HIP(hipMemcpyAsync(b->slots_h.data(), b->slots_d, sizeof(GraphSlot) * b->G, hipMemcpyDeviceToHost,
                           b->stream));
    MFB_HIP(hipStreamSynchronize(b->stream));
    mf_status rc = MF_OK;
    for (int i = 0; i < b->G; ++i) {
        values[i] = b->slots_h[i].value;
        if (b->slots_h[i].status != 0) rc = MF_ERR_NOT_CONVERGED;
    }
    return rc;
}

// Around the solve launch of a call: while profiling, the partial byte sums
// start at zero and events bracket the launch.
mf_status prof_begin(mf_batch* b) {
    if (!b->prof) return MF_OK;
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(b->bytes_part), 0, 2 * (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS,
                        b->stream);
    MFB_HIP(hipEventRecord(b->ev[0], b->stream));
    return MF_OK;
}

mf_status prof_end(mf_batch* b) {
    if (!b->prof) return MF_OK;
    MFB_HIP(hipEventRecord(b->ev[1], b->stream));
    b->bytes_h.resize((size_t)mf::KC_NCLASS * mf::BYTES_SLOTS);
    MFB_HIP(hipMemcpyAsync(b->bytes_h.data(), b->bytes_part, sizeof(unsigned long long) * b->bytes_h.size(),
                           hipMemcpyDeviceToHost, b->stream));
    MFB_HIP(hipStreamSynchronize(b->stream));
    float ms = 0;
    MFB_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
    b->kernel_ms = ms;
    double sum = 0;
    for (unsigned long long x : b->bytes_h) sum += (double)x;
    b->kernel_bytes = sum;
    return MF_OK;
}

struct Clock {
    mf_batch* b;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    explicit Clock(mf_batch* bb) : b(bb) {}
    ~Clock() {
        b->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};


// Tuning fields from resolved options; KC per graph defaults to round(m/n).
void apply_tuning(mf_batch* b, const mf::Tuning& t) {
    b->tune = t.gr;
    b->tune.lds = 0;
    b->round_div = t.round_div;
    b->bin0 = t.bin0;
    b->bin1 = t.bin1;
    b->block = t.batch_block;
    b->kc_option = t.kc_option;
    b->long_cycles = t.long_cycles;
    for (int i = 0; i < b->G; ++i) {
        int64_t kc = t.kc_option > 0 ? t.kc_option : (b->m_unique[i] + b->n[i] / 2) / b->n[i];
        b->kc[i] = (int32_t)std::max<int64_t>(1, kc);
    }
}

// Slot and queue bases of every graph for the current slot counts.
void set_slot_bases(mf_batch* b) {
    b->total_s = 0;
    b->total_q = 0;
    for (int i = 0; i < b->G; ++i) {
        b->sbase[i] = b->total_s;
        b->qbase[i] = b->total_q;
        b->total_s += b->slots[i];
        b->total_q += 2 * ((int64_t)b->n[i] + b->slots[i] / mf::GR_CHUNK + 64);
    }
}

// (Re)allocates the slot-sized pools and the BFS queues, then uploads every
// graph's rows and slots from hb (slot indices local to each graph, made
// pool-global here).  res: residual per slot of each graph, or null for
// res = cap (zero flow).  The vertex-sized pools must exist already.
mf_status upload_slots(mf_batch* b, const std::vector<mf::HostBiCSR>& hb,
                       const std::vector<std::vector<int32_t>>* res) {
    const int G = b->G;
    const int64_t V = b->total_v, SS = b->total_s;
    bfree(b->cr); bfree(b->rev); bfree(b->cap); bfree(b->capsum); bfree(b->win); bfree(b->q);
    if (balloc(&b->cr, SS) || balloc(&b->rev, SS) || balloc(&b->cap, SS) || balloc(&b->capsum, SS) ||
        balloc(&b->win, SS) || balloc(&b->q, b->total_q))
        return MF_ERR_OUT_OF_MEMORY;
    std::vector<int32_t> rp((size_t)b->total_rp), rl((size_t)V), rs((size_t)V), rv((size_t)SS),
        cp((size_t)SS), cs((size_t)SS, 0);
    std::vector<int2> crh((size_t)SS);
    b->used.assign((size_t)G, 0);
    for (int i = 0; i < G; ++i) {
        const mf::HostBiCSR& x = hb[(size_t)i];
        const int32_t ni = b->n[i];
        const int64_t sb = b->sbase[i];
        for (int32_t v = 0; v <= ni; ++v) rp[(size_t)(b->rpbase[i] + v)] = (int32_t)(sb + x.row_ptr[(size_t)v]);
        for (int32_t v = 0; v < ni; ++v) {
            rl[(size_t)(b->vbase[i] + v)] = x.row_len[(size_t)v];
            rs[(size_t)(b->vbase[i] + v)] = x.row_sorted[(size_t)v];
            b->used[(size_t)i] += x.row_len[(size_t)v];
        }
        const std::vector<int32_t>* r = res ? &(*res)[(size_t)i] : nullptr;
        for (int64_t j = 0; j < b->slots[i]; ++j) {
            int32_t c = x.cap[(size_t)j];
            crh[(size_t)(sb + j)] = make_int2(x.col[(size_t)j], r ? (*r)[(size_t)j] : c);
            cp[(size_t)(sb + j)] = c;
            int32_t rj = x.rev[(size_t)j];
            rv[(size_t)(sb + j)] = rj >= 0 ? (int32_t)(sb + rj) : -1;
            if (rj >= 0) cs[(size_t)(sb + j)] = c + x.cap[(size_t)rj];
        }
    }
    hipStream_t st = b->stream;
    if (hipMemcpyAsync(b->row_ptr, rp.data(), 4 * rp.size(), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(b->row_len, rl.data(), 4 * rl.size(), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(b->row_sorted, rs.data(), 4 * rs.size(), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(b->cr, crh.data(), 8 * crh.size(), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(b->rev, rv.data(), 4 * rv.size(), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(b->cap, cp.data(), 4 * cp.size(), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(b->capsum, cs.data(), 4 * cs.size(), hipMemcpyHostToDevice, st))
        return MF_ERR_DEVICE;
    mf::launch_fill_i32(b->win, -1, SS, st);
    // the host images are freed on return: wait for the copies
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return MF_ERR_DEVICE;
    return MF_OK;
}

// Per-graph views over the pools (results of the last launch are kept), and
// the solve order (largest graphs first, so that the long solves start
// early), uploaded.
mf_status upload_views(mf_batch* b) {
    const int G = b->G;
    b->slots_h.resize((size_t)G);
    for (int i = 0; i < G; ++i) {
        GraphSlot& S = b->slots_h[(size_t)i];
        const int32_t ni = b->n[i];
        mf::DevGraph& g = S.g;
        g.n = ni;
        g.s = b->s_h[(size_t)i];
        g.t = b->t_h[(size_t)i];
        g.root = g.t;
        g.pinned = g.s;
        g.row_ptr = b->row_ptr + b->rpbase[i];
        g.row_len = b->row_len + b->vbase[i];
        g.row_sorted = b->row_sorted + b->vbase[i];
        g.cr = b->cr;
        g.rev = b->rev;
        g.cap = b->cap;
        g.capsum = b->capsum;
        g.e = b->e + b->vbase[i];
        g.h = b->h + b->vbase[i];
        g.used_slots = b->used[(size_t)i];
        g.nslots = nullptr;  // the batched kernels keep used_slots in the device-resident view
        g.halt = nullptr;
        g.bfs_cap = 0;
        g.h_prev = nullptr;
        g.bytes_part = b->bytes_part;
        g.count_bytes = b->prof ? 1 : 0;
        g.bin0_max = b->bin0;
        g.bin1_max = b->bin1;
        g.side = nullptr;
        g.side_keep = 0;
        g.act = nullptr;
        g.act_cnt = nullptr;
        g.relab = nullptr;
        g.act_cap = 0;
        int64_t qc = (int64_t)ni + b->slots[i] / mf::GR_CHUNK + 64;
        S.q0 = b->q + b->qbase[i];
        S.q1 = S.q0 + qc;
        S.wl0 = b->wl + 3 * b->vbase[i];
        S.wl1 = S.wl0 + ni;
        S.wl2 = S.wl1 + ni;
        S.bits.nwords = (ni + 31) / 32;
        S.bits.visited = b->bits + b->bbase[i];
        S.bits.fb = S.bits.visited + S.bits.nwords;
        S.ctr = b->ctr + i;
        S.kc = b->kc[i];
        S.kc_long = std::min(b->kc[i], b->long_cycles);
        S.warm = b->opt.cold_start ? 0 : 1;
        S.round_div = b->round_div;
        S.max_iter = b->opt.max_iterations > 0 ? b->opt.max_iterations : 4 * (int64_t)ni + 1000;
    }
    std::vector<int32_t> order((size_t)G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return b->slots[a] > b->slots[c]; });
    if (hipMemcpy(b->slots_d, b->slots_h.data(), sizeof(GraphSlot) * G, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->order_d, order.data(), 4 * (size_t)G, hipMemcpyHostToDevice) != hipSuccess)
        return MF_ERR_DEVICE;
    return MF_OK;
}

// A batch's inserts did not fit the free slots of some rows: re-lay the rows
// of the graphs flagged in `grow` on the device with room for need[] more
// (residuals, excesses and heights are kept), move every graph to its new
// place in the pools and rebuild the views.  A device failure leaves the
// batch poisoned.
mf_status relayout_pool(mf_batch* b, const int32_t* need_d, const std::vector<char>& grow) {
    const int G = b->G;
    const int64_t V = b->total_v;
    hipStream_t st = b->stream;
    if (!b->gid_d) {
        std::vector<int32_t> gid((size_t)V);
        for (int i = 0; i < G; ++i)
            std::fill(gid.begin() + b->vbase[i], gid.begin() + b->vbase[i] + b->n[i], i);
        if (balloc(&b->gid_d, V) || balloc(&b->vbase_d, G) || balloc(&b->grow_d, G)) return MF_ERR_OUT_OF_MEMORY;
        MFB_HIP(hipMemcpyAsync(b->gid_d, gid.data(), 4 * (size_t)V, hipMemcpyHostToDevice, st));
        MFB_HIP(hipMemcpyAsync(b->vbase_d, b->vbase.data(), 8 * (size_t)G, hipMemcpyHostToDevice, st));
        MFB_HIP(hipStreamSynchronize(st));
    }
    std::vector<uint8_t> gr(grow.begin(), grow.end());
    MFB_HIP(hipMemcpyAsync(b->grow_d, gr.data(), (size_t)G, hipMemcpyHostToDevice, st));
    for (int i = 0; i < G; ++i) b->used[(size_t)i] = b->slots_h[(size_t)i].g.used_slots;
    mf::RelayoutPlan p{};
    p.V = (int32_t)V;
    p.row_ptr = b->row_ptr;
    p.row_len = b->row_len;
    p.row_sorted = b->row_sorted;
    p.need = need_d;
    p.gid = b->gid_d;
    p.vbase = b->vbase_d;
    p.grow = b->grow_d;
    p.slack_min = b->slack_min;
    p.slack_pct = b->slack_pct;
    p.slack_shift = std::min(b->relayouts + 1, 3);  // as for single graphs
    mf::SlotArrays a{b->cr, b->rev, b->cap, b->capsum};
    int64_t S = 0;
    mf_status rc = mf::relayout_device(p, &a, b->total_s, &S, b->row_ptr, b->row_sorted, st, b->mem);
    if (rc != MF_OK) {
        if (rc == MF_ERR_DEVICE) b->poisoned = true;
        return rc;
    }
    b->cr = a.cr;
    b->rev = a.rev;
    b->cap = a.cap;
    b->capsum = a.capsum;
    // per-graph slot counts from the new row pointers (graphs stay in order)
    std::vector<int32_t> rp((size_t)b->total_rp);
    MFB_HIP(hipMemcpyAsync(rp.data(), b->row_ptr, 4 * rp.size(), hipMemcpyDeviceToHost, st));
    MFB_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < G; ++i) b->slots[i] = (int64_t)rp[(size_t)(b->rpbase[i] + b->n[i])] - rp[(size_t)b->rpbase[i]];
    set_slot_bases(b);
    bfree(b->win);
    bfree(b->q);
    if (b->total_s != S || balloc(&b->win, S) || balloc(&b->q, b->total_q)) {
        b->poisoned = true;
        return MF_ERR_DEVICE;
    }
    mf::launch_fill_i32(b->win, -1, S, st);
    MFB_HIP(hipGetLastError());
    rc = upload_views(b);
    if (rc != MF_OK) {
        b->poisoned = true;
        return rc;
    }
    b->relayouts++;
    return MF_OK;
}

}  // namespace

extern "C" {

mf_status mf_batch_load(int32_t num_graphs, const int32_t* n, const int64_t* edge_offset,
                        const int32_t* src, const int32_t* dst, const int32_t* cap, const int32_t* s,
                        const int32_t* t, const mf_options* opt, mf_batch** out) {
    if (!out) return MF_ERR_INVALID;
    *out = nullptr;
    if (num_graphs < 1 || !n || !edge_offset || !s || !t) return MF_ERR_INVALID;
    mf_options o;
    mf_default_options(&o);
    if (opt) {
        if (opt->struct_size != sizeof(mf_options)) return MF_ERR_INVALID;
        o = *opt;
    }
    if (edge_offset[0] != 0) return MF_ERR_INVALID;
    for (int i = 0; i < num_graphs; ++i)
        if (edge_offset[i + 1] < edge_offset[i]) return MF_ERR_INVALID;
    int32_t slack_min = o.insert_slack_min > 0 ? o.insert_slack_min : 8;
    int32_t slack_pct = o.insert_slack_pct > 0 ? o.insert_slack_pct : 12;
    mf::Tuning tuning;
    if (mf::resolve_tuning(o, &tuning) != MF_OK) return MF_ERR_INVALID;
    // validate and build every graph on the host first: nothing is allocated on failure
    std::vector<mf::HostBiCSR> hb((size_t)num_graphs);
    for (int i = 0; i < num_graphs; ++i) {
        int64_t e0 = edge_offset[i], m = edge_offset[i + 1] - e0;
        mf_status rc = mf::build_bicsr(n[i], m, m ? src + e0 : nullptr, m ? dst + e0 : nullptr,
                                       m ? cap + e0 : nullptr, s[i], t[i], slack_min, slack_pct, &hb[(size_t)i]);
        if (rc != MF_OK) return rc;
    }
    if ((o.alloc == nullptr) != (o.free == nullptr)) return MF_ERR_INVALID;
    mf_batch* b = new (std::nothrow) mf_batch();
    if (!b) return MF_ERR_OUT_OF_MEMORY;
    b->mem.alloc_fn = o.alloc;
    b->mem.free_fn = o.free;
    b->mem.ctx = o.alloc_ctx;
    UseAllocator use(b->mem);
    auto fail = [&](mf_status r) {
        free_batch(b);
        if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return r;
    };
    b->G = num_graphs;
    b->opt = o;
    int dev = o.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(MF_ERR_DEVICE);
    if (hipSetDevice(dev) != hipSuccess) return fail(MF_ERR_DEVICE);
    b->device = dev;
    if (o.stream) {
        b->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return fail(MF_ERR_DEVICE);
        b->own_stream = true;
    }
    const int G = num_graphs;
    b->slack_min = slack_min;
    b->slack_pct = slack_pct;
    b->s_h.assign(s, s + G);
    b->t_h.assign(t, t + G);
    b->n.resize(G); b->kc.resize(G); b->vbase.resize(G); b->rpbase.resize(G); b->sbase.resize(G);
    b->slots.resize(G); b->bbase.resize(G); b->qbase.resize(G); b->m_unique.resize(G);
    for (int i = 0; i < G; ++i) {
        const mf::HostBiCSR& x = hb[(size_t)i];
        b->n[i] = n[i];
        b->m_unique[i] = x.m_unique;
        b->vbase[i] = b->total_v;
        b->rpbase[i] = b->total_rp;
        b->slots[i] = x.row_ptr[(size_t)n[i]];
        b->bbase[i] = b->total_b;
        b->total_v += n[i];
        b->total_rp += n[i] + 1;
        b->total_b += 4 * (int64_t)((n[i] + 31) / 32);
    }
    apply_tuning(b, tuning);
    set_slot_bases(b);
    if (b->total_s > INT_MAX || b->total_v > INT_MAX) return fail(MF_ERR_OVERFLOW);
    const int64_t V = b->total_v;
    if (balloc(&b->row_ptr, b->total_rp) || balloc(&b->row_len, V) || balloc(&b->row_sorted, V) ||
        balloc(&b->need, V) || balloc(&b->e, V) || balloc(&b->h, V) || balloc(&b->bits, b->total_b) ||
        balloc(&b->wl, 3 * V) || balloc(&b->ctr, G) ||
        balloc(&b->bytes_part, (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS) || balloc(&b->slots_d, G) ||
        balloc(&b->order_d, G))
        return fail(MF_ERR_OUT_OF_MEMORY);
    hipStream_t st = b->stream;
    mf::launch_fill_i32(b->need, 0, V, st);
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(b->e), 0, 2 * V, st);
    mf::launch_fill_i32(b->h, 0, V, st);
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(b->bytes_part), 0, 2 * (int64_t)mf::KC_NCLASS * mf::BYTES_SLOTS,
                        st);
    mf::launch_fill_i32(reinterpret_cast<int32_t*>(b->ctr), 0, (int64_t)G * sizeof(DevCounters) / 4, st);
    mf_status rc = upload_slots(b, hb, nullptr);
    if (rc != MF_OK) return fail(rc);
    hb.clear();
    hb.shrink_to_fit();
    rc = upload_views(b);
    if (rc != MF_OK) return fail(rc);
    *out = b;
    return MF_OK;
}

mf_status mf_batch_maxflow(mf_batch* b, int64_t* values) {
    if (!b || !values) return MF_ERR_INVALID;
    if (b->poisoned) return MF_ERR_DEVICE;
    if (hipSetDevice(b->device) != hipSuccess) return MF_ERR_DEVICE;
    Clock clock(b);
    b->solved = false;
    mf_status rc = prof_begin(b);
    if (rc != MF_OK) return rc;
    mf::launch_batch_solve(b->slots_d, b->order_d, b->G, 0, b->tune, b->block, b->stream);
    MFB_HIP(hipGetLastError());
    rc = prof_end(b);
    if (rc != MF_OK) return rc;
    rc = read_results(b, values);
    if (rc == MF_OK) b->solved = true;
    return rc;
}

mf_status mf_batch_apply(mf_batch* b, const int64_t* update_offset, const mf_update* upd, int64_t* values) {
    if (!b || !update_offset || !values) return MF_ERR_INVALID;
    if (b->poisoned) return MF_ERR_DEVICE;
    if (!b->solved) return MF_ERR_STATE;
    const int G = b->G;
    if (update_offset[0] != 0) return MF_ERR_INVALID;
    for (int i = 0; i < G; ++i)
        if (update_offset[i + 1] < update_offset[i] || update_offset[i + 1] - update_offset[i] > INT_MAX / 2)
            return MF_ERR_INVALID;
    const int64_t K = update_offset[G];
    if (K > 0 && !upd) return MF_ERR_INVALID;
    if (hipSetDevice(b->device) != hipSuccess) return MF_ERR_DEVICE;
    Clock clock(b);
    UseAllocator use(b->mem);
    hipStream_t st = b->stream;
    // scratch: updates, per-update slots, one hash table per graph
    std::vector<int64_t> toff((size_t)G + 1, 0);
    std::vector<int32_t> tcap((size_t)G);
    for (int i = 0; i < G; ++i) {
        int64_t k = update_offset[i + 1] - update_offset[i];
        int32_t c = 16;
        while (c < 2 * k) c *= 2;
        tcap[(size_t)i] = c;
        toff[(size_t)i + 1] = toff[(size_t)i] + c;
    }
    if (K > b->upd_cap) {
        MFB_HIP(hipStreamSynchronize(st));
        bfree(b->upd_d); bfree(b->slot_of); bfree(b->touched);
        if (balloc(&b->upd_d, K) || balloc(&b->slot_of, K) || balloc(&b->touched, K)) {
            b->upd_cap = 0;
            return MF_ERR_OUT_OF_MEMORY;
        }
        b->upd_cap = K;
    }
    if (toff[(size_t)G] > b->tab_cap) {
        MFB_HIP(hipStreamSynchronize(st));
        bfree(b->tkey); bfree(b->twin); bfree(b->tslot);
        int64_t c = toff[(size_t)G];
        if (balloc(&b->tkey, c) || balloc(&b->twin, 2 * c) || balloc(&b->tslot, 2 * c)) {
            b->tab_cap = 0;
            return MF_ERR_OUT_OF_MEMORY;
        }
        mf::launch_fill_i32(reinterpret_cast<int32_t*>(b->tkey), -1, 2 * c, st);
        mf::launch_fill_i32(b->twin, -1, 2 * c, st);
        b->tab_cap = c;
    }
    if (!b->gu_d && balloc(&b->gu_d, G)) return MF_ERR_OUT_OF_MEMORY;
    if (K > 0) MFB_HIP(hipMemcpyAsync(b->upd_d, upd, sizeof(mf_update) * (size_t)K, hipMemcpyHostToDevice, st));
    b->ctr_h.resize((size_t)G);
    for (int attempt = 0;; ++attempt) {
        bool relay_fail = false;
        std::vector<GraphUpdates> gu((size_t)G);
        for (int i = 0; i < G; ++i) {
            GraphUpdates& U = gu[(size_t)i];
            int64_t o0 = update_offset[i];
            U.upd = b->upd_d + o0;
            U.k = (int32_t)(update_offset[i + 1] - o0);
            U.slot_of = b->slot_of + o0;
            U.touched = b->touched + o0;
            U.win = b->win;
            U.need = b->need + b->vbase[i];
            U.tb.key = b->tkey + toff[(size_t)i];
            U.tb.win = b->twin + 2 * toff[(size_t)i];
            U.tb.slot = b->tslot + 2 * toff[(size_t)i];
            U.tb.capacity = tcap[(size_t)i];
        }
        MFB_HIP(hipMemcpyAsync(b->gu_d, gu.data(), sizeof(GraphUpdates) * (size_t)G, hipMemcpyHostToDevice, st));
        mf::launch_batch_locate_multi(b->slots_d, b->gu_d, G, st);
        MFB_HIP(hipGetLastError());
        MFB_HIP(hipMemcpyAsync(b->ctr_h.data(), b->ctr, sizeof(DevCounters) * (size_t)G, hipMemcpyDeviceToHost, st));
        MFB_HIP(hipStreamSynchronize(st));
        bool err = false, ovf = false, slack = false;
        std::vector<char> grow((size_t)G, 0);
        for (int i = 0; i < G; ++i) {
            err |= b->ctr_h[(size_t)i].err != 0;
            ovf |= b->ctr_h[(size_t)i].cap_overflow != 0;
            grow[(size_t)i] = b->ctr_h[(size_t)i].overflow != 0;
            slack |= grow[(size_t)i] != 0;
        }
        if (!err && !ovf && !slack) break;
        // nothing was changed yet.  Rows without room for their inserts: keep
        // need[] (the per-row demand), return the scratch to idle, re-lay
        // those graphs and locate again.
        const bool relay = !err && !ovf && attempt < 2;
        if (relay) {
            if (!b->need_copy && balloc(&b->need_copy, b->total_v)) relay_fail = true;
            else MFB_HIP(hipMemcpyAsync(b->need_copy, b->need, 4 * (size_t)b->total_v, hipMemcpyDeviceToDevice, st));
        }
        mf::launch_batch_cleanup_multi(b->gu_d, G, st);
        MFB_HIP(hipGetLastError());
        MFB_HIP(hipStreamSynchronize(st));
        if (err) return MF_ERR_INVALID;
        if (ovf || !relay) return MF_ERR_OVERFLOW;
        if (relay_fail) return MF_ERR_OUT_OF_MEMORY;
        mf_status rc = relayout_pool(b, b->need_copy, grow);
        if (rc != MF_OK) return rc;
    }
    b->solved = false;
    mf_status rc = prof_begin(b);
    if (rc != MF_OK) return rc;
    mf::launch_batch_repair_multi(b->slots_d, b->gu_d, b->order_d, G, b->tune, b->block, st);
    MFB_HIP(hipGetLastError());
    rc = prof_end(b);
    if (rc != MF_OK) return rc;
    rc = read_results(b, values);
    if (rc == MF_OK) b->solved = true;
    return rc;
}

mf_status mf_batch_tune(mf_batch* b, const mf_options* opt) {
    if (!b || !opt || opt->struct_size != sizeof(mf_options)) return MF_ERR_INVALID;
    if (b->poisoned) return MF_ERR_DEVICE;
    mf::Tuning t;
    if (mf::resolve_tuning(*opt, &t) != MF_OK) return MF_ERR_INVALID;
    if (hipSetDevice(b->device) != hipSuccess) return MF_ERR_DEVICE;
    MFB_HIP(hipStreamSynchronize(b->stream));
    apply_tuning(b, t);
    return upload_views(b);
}

mf_status mf_batch_info(const mf_batch* b, int32_t* iterations, double* last_ms) {
    if (!b) return MF_ERR_INVALID;
    if (iterations)
        for (int i = 0; i < b->G; ++i) iterations[i] = b->slots_h[(size_t)i].iterations;
    if (last_ms) *last_ms = b->last_ms;
    return MF_OK;
}

mf_status mf_batch_profile(mf_batch* b, int32_t on) {
    if (!b) return MF_ERR_INVALID;
    if (b->poisoned) return MF_ERR_DEVICE;
    if (hipSetDevice(b->device) != hipSuccess) return MF_ERR_DEVICE;
    MFB_HIP(hipStreamSynchronize(b->stream));
    for (auto& e : b->ev)
        if (!e) MFB_HIP(hipEventCreate(&e));
    b->prof = on != 0;
    b->kernel_ms = b->kernel_bytes = 0;
    return upload_views(b);
}

mf_status mf_batch_kernel_stats(const mf_batch* b, double* kernel_ms, double* alg_bytes) {
    if (!b) return MF_ERR_INVALID;
    if (kernel_ms) *kernel_ms = b->kernel_ms;
    if (alg_bytes) *alg_bytes = b->kernel_bytes;
    return MF_OK;
}

void mf_batch_free(mf_batch* b) {
    if (!b) return;
    UseAllocator use(b->mem);
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    for (auto e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
