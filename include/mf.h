/*
 * mf.h -- C ABI of the MI355X (gfx950) dynamic max-flow library.
 *
 * The library computes the maximum s-t flow value of a capacitated directed
 * graph (paper Section 2.1) with the GPU push-relabel loop of Section 3
 * (Algorithms 1-4: preflow initialisation, push-relabel kernel,
 * remove-invalid-edges kernel, backward-BFS global relabel) and repairs it
 * after a batch of capacity updates with the dynamic algorithm of Section 4
 * (Algorithms 5-6: apply capacity deltas, send back over-capacity flow,
 * re-saturate the source, global relabel that treats deficient vertices as
 * extra sinks, then the same push-relabel loop).  The residual graph is the
 * Bi-CSR of Section 5.1: every vertex row holds both its out- and in-
 * neighbours, absent reverse edges as zero-capacity entries, and every entry
 * knows the index of its reverse entry.
 *
 * Conventions for every call
 *   - Integers are fixed-width.  Capacities are int32 >= 0; flow values and
 *     excesses are exact int64.  There is no floating point in the method.
 *   - Host pointers passed in are only read during the call (the library
 *     copies what it keeps); output buffers are owned by the caller.
 *   - A graph handle owns all device memory of its graph until
 *     mf_graph_free.  One handle must not be used by two threads at once;
 *     distinct handles are independent.
 *   - Calls are synchronous with respect to their outputs: when a call
 *     returns, its host outputs are written.
 *   - Inputs are validated before anything is changed: on every error other
 *     than MF_ERR_DEVICE the graph is left exactly as it was.  After
 *     MF_ERR_DEVICE the handle only accepts mf_graph_free.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf_graph mf_graph;

typedef enum mf_status {
    MF_OK = 0,
    MF_ERR_INVALID = 1,        /* bad argument: ids out of range, u == v, s == t, cap < 0, n < 2, k < 0, NULL */
    MF_ERR_OUT_OF_MEMORY = 2,  /* a device or host allocation failed; the graph is unchanged */
    MF_ERR_OVERFLOW = 3,       /* c(u,v) + c(v,u) of a merged pair exceeds INT32_MAX, or too many slots */
    MF_ERR_DEVICE = 4,         /* a HIP call failed; the handle is unusable */
    MF_ERR_NOT_CONVERGED = 5,  /* the global-relabel iteration cap was reached */
    MF_ERR_STATE = 6           /* call order: a repair, cut or flow before the first mf_maxflow */
} mf_status;

/* Options.  Zero-initialise, set struct_size = sizeof(mf_options), or call
 * mf_default_options.  Fields left 0 take the default shown. */
typedef struct mf_options {
    uint32_t struct_size;
    int32_t device;            /* HIP device ordinal; default: the current device */
    void* stream;              /* hipStream_t to launch on (e.g. a torch stream); NULL: a library stream */
    int32_t kernel_cycles;     /* push/relabel cycles per vertex per launch (Algorithm 2's
                                  KERNEL_CYCLES); <= 0: round(m/n), at least 1 (Section 6.1) */
    int32_t topology_driven;   /* 1: one worker per vertex for push-relabel and remove-invalid-
                                  edges; 0 (default): active-vertex worklist (Section 5.2, O1) */
    int32_t insert_slack_min;  /* free slots kept per row for inserted pairs; <= 0: 8 */
    int32_t insert_slack_pct;  /* plus this percentage of the row's length; <= 0: 12 */
    int64_t max_iterations;    /* cap on global relabels per call; <= 0: 4n + 1000 */
    int32_t cold_start;        /* 0 (default): a repair first runs one push-relabel and remove-
                                  invalid-edges sweep on the heights left by the previous solve, then
                                  the loop; 1: the loop right away, global relabel first (Algorithm 5
                                  as printed).  Both return the same value. */
    int32_t relabel_mode;      /* 0 (default): one launch per BFS level; 1: the whole global
                                  relabel and worklist build in one cooperative launch with a grid
                                  barrier per level (falls back to 0 where unsupported) */
    /* tuning (mf_graph_tune / mf_batch_tune change them on a live handle); none
     * changes a result */
    int32_t bfs_alpha;         /* a BFS level goes bottom-up when its frontier's slots times alpha
                                  exceed the unvisited slots ...; 0: 14, < 0: never bottom-up */
    int32_t bfs_beta;          /* ... and its frontier vertices times beta exceed n; <= 0: 64 */
    int32_t round_div;         /* push-relabel rounds per global relabel: BFS depth / round_div,
                                  at least 1; <= 0: 4 */
    int32_t bin_thread_max;    /* active rows up to this many slots get one thread ...; <= 0: 16 */
    int32_t bin_wave_max;      /* ... up to this many one 64-lane wave, longer ones a workgroup;
                                  <= 0: 512 */
    int32_t batch_block;       /* mf_batch_*: threads per graph, 256, 512 or 1024; 0: 1024 */
    int32_t push_pull;         /* 1: Section 5.2's O2 -- mf_maxflow also saturates the sink's
                                  in-edges first (static push-pull); a repair saturates the previous
                                  min cut again and runs push-relabel on its sink side and pull-
                                  relabel on its source side at the same time on two streams,
                                  before the ordinary loop.  0 (default): off.  Same values. */
    /* Device memory: every buffer a handle (or batch) owns is taken from
     * alloc(bytes, alloc_ctx) and given back with free(ptr, alloc_ctx), e.g. a
     * framework's caching allocator (launch the handle on that framework's
     * stream then).  Both NULL (default): hipMalloc / hipFree.  Setting only
     * one is MF_ERR_INVALID.  alloc returns NULL when it has no memory. */
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* alloc_ctx;
    int32_t long_row_cycles;   /* tuning: push/relabel cycles per launch for the rows a workgroup
                                  takes (longer than bin_wave_max slots), at most kernel_cycles;
                                  <= 0: 1.  Their excess left over waits for the next round, so a
                                  hub's repeated full-row passes do not hold up the launch
                                  (in mf_batch_*, the graph's other rows). */
    /* Loop and relabel settings of a single-graph handle (mf_graph_tune changes
     * them on a live handle too).  None changes a result.  0 takes the
     * default; on/off switches take 1 = on, -1 = off. */
    int32_t bfs_first_chunk;   /* BFS levels launched before the host first checks whether the
                                  BFS is over (a relabel of depth d launches max(this, d + 1));
                                  <= 0: 7 */
    int32_t bfs_narrow_slots;  /* frontiers of at most this many slots run in one workgroup, many
                                  levels per launch; 0: 4096, < 0: never */
    int32_t bfs_medium_slots;  /* larger frontiers up to this many slots run in one cooperative
                                  launch of bfs_medium_blocks workgroups with a grid barrier per
                                  level; 0: 65536, < 0: never (also where cooperative launch is
                                  unsupported) */
    int32_t bfs_medium_blocks; /* 0: 16 */
    int32_t bfs_level_blocks;  /* workgroups of one multi-block BFS level launch; 0: four per
                                  compute unit */
    int32_t bfs_bottom_up;     /* bottom-up level variant: 0 a thread per unvisited row, four slot
                                  loads in flight; 1 the same with eight; 2 slot-parallel over
                                  the unvisited rows (no early exit per row) */
    int32_t bfs_lds_bitmap;    /* 1: top-down levels of at least bfs_stage_min frontier entries read
                                  the visited bitmap from a copy in LDS, where it fits */
    int32_t bfs_stage_min;     /* 0: 1024 */
    int32_t round_min;         /* push-relabel rounds per global relabel: at least this many
                                  (and BFS depth / round_div); 0: 2 */
    int32_t round_max;         /* ... and at most this many; 0: 4096 */
    int32_t round_scan;        /* 1: every round's worklist comes from a scan of every vertex;
                                  0: from the last worklist plus the round's activations */
    int32_t queue_rounds;      /* -1: the worklist build and the first two rounds are not queued
                                  behind the relabel's first chunk of levels (three read-backs
                                  per iteration instead of one) */
    int32_t pipeline;          /* -1: on shallow graphs the next iteration is not queued before
                                  the host reads the last one's counters */
    int32_t graph_capture;     /* 1: every pipelined iteration is one launch of a HIP graph
                                  captured once per handle (and again when a relayout, restore
                                  or tuning changes what it bakes in); 0 (default) or -1: its
                                  kernels are launched one by one, which measured faster */
    int32_t trace;             /* 1: every BFS level (one per launch) and every round printed on
                                  stderr, for diagnosis; slow */
    int32_t round_narrow;      /* rounds between relabels whose worklist holds at most this many
                                  vertices (none above bin_wave_max slots) run in one workgroup,
                                  many rounds per launch, and such a relabel buys at least 8 of
                                  them (they stop when the list empties); 0: 2048, < 0: never */
    int32_t bfs_cap;           /* 0 (default) or 1: a solve's relabels after its first one, when no
                                  deficient vertex sits above height 0, stop once every vertex with
                                  excess below |V| has its height; a vertex not reached keeps
                                  max(depth + 1, its old height) (a valid labelling, not distances;
                                  mf_min_cut relabels first).  -1: every relabel runs to the end */
} mf_options;

/* One update of a batch: set c(u,v) := cap.  cap == 0 deletes the edge (its
 * slot stays, with capacity 0); an absent pair is inserted.  Within one
 * batch the last update of a pair wins.  (Section 4.1: a batch is a set of
 * edges with their new capacities, higher or lower than before.) */
typedef struct mf_update {
    int32_t u, v, cap;
} mf_update;

typedef struct mf_stats {
    int64_t n;                 /* vertices */
    int64_t pairs;             /* directed pairs (u,v) with a Bi-CSR entry in row u (cap may be 0) */
    int64_t slots;             /* Bi-CSR entries in use (one per such pair) */
    int64_t slot_capacity;     /* Bi-CSR entries allocated, including insertion slack */
    int64_t device_bytes;      /* device memory held by the handle */
    int32_t kernel_cycles;     /* KC in use */
    int32_t relayouts;         /* times insertion slack ran out and the rows were re-laid */
    /* counters of the last mf_maxflow / mf_apply_batch call */
    int64_t last_iterations;   /* global relabels (loop iterations) */
    int64_t last_bfs_levels;   /* BFS level launches summed over its global relabels */
    int64_t last_active_sum;   /* sum over iterations of the worklist size */
    int64_t last_new_pairs;    /* pairs inserted by the last batch */
    double last_ms;            /* host wall time of the call */
    /* per-kernel device time over the calls since mf_profile (HIP events on the
     * library's stream); index: 0 global-relabel multi-block BFS level, 1 push-relabel,
     * 2 remove-invalid-edges, 3 worklist build, 4 batch kernels, 5 reset and source
     * saturation, 6 global-relabel seeding and one-workgroup thin-frontier levels */
    double kernel_ms[8];
    int64_t kernel_launches[8];
    /* algorithmic bytes the kernels of each class had to move over the same calls,
     * from device-side counters (Bi-CSR slots and vertex words actually visited) */
    double kernel_bytes[8];
    int64_t last_rounds;       /* push-relabel rounds of the last call (two or more per global relabel
                                  that leaves active vertices, unless a round empties the worklist) */
    int64_t last_capped_relabels; /* global relabels of the last call whose BFS stopped before the end
                                  (bfs_cap) */
} mf_stats;

/* Fill *opt with the defaults. */
void mf_default_options(mf_options* opt);

/* Human-readable name of a status code (static storage). */
const char* mf_status_string(mf_status status);

/* Load a graph (Section 2.1: directed G=(V,E), capacities c >= 0, source s,
 * sink t) and build its device Bi-CSR (Section 5.1).
 *   n        number of vertices, >= 2; vertices are 0..n-1
 *   m        number of edges, >= 0
 *   src,dst  int32[m] endpoints, host memory; u == v is rejected
 *   cap      int32[m] capacities >= 0, host memory; repeated (u,v) pairs add up
 *   s, t     source and sink, distinct
 *   opt      NULL for defaults
 *   out      receives the handle
 * No flow is computed; the residual graph starts at zero flow.
 * Errors: MF_ERR_INVALID, MF_ERR_OVERFLOW (a merged pair's c(u,v)+c(v,u) above
 * INT32_MAX), MF_ERR_OUT_OF_MEMORY, MF_ERR_DEVICE. */
mf_status mf_graph_load(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* cap, int32_t s, int32_t t, const mf_options* opt,
                        mf_graph** out);

/* Maximum flow value of the current capacities from zero flow: Algorithm 1
 * (initialise, saturate the source, loop {backward BFS, push-relabel kernel,
 * remove-invalid-edges kernel} while active vertices remain).  The loop stops
 * when no active vertex is left under a valid labelling -- right after a
 * global relabel, or after a push-relabel plus remove-invalid-edges round,
 * which keeps the labelling valid -- and *value = e(t) plus the
 * (non-positive) excess of every deficient vertex.
 * Leaves the residual graph, excesses and heights on the device for repairs.
 * The value is final on return; the handle's stream may still be running the
 * launches of one more iteration (queued before the last one's counters were
 * read), which find the loop over on the device and leave at once.  Every
 * later call on the handle is ordered after them on that stream.
 * Errors: MF_ERR_INVALID (NULL), MF_ERR_NOT_CONVERGED, MF_ERR_DEVICE. */
mf_status mf_maxflow(mf_graph* g, int64_t* value);

/* Apply a batch of k updates held in HOST memory and return the new maximum
 * flow value, repairing the retained state as Algorithm 5 does: add each
 * capacity change to the residual, send back flow above a lowered capacity
 * (changing the two endpoints' excesses), saturate the source again, then
 * run the loop with t and every deficient vertex as sinks (Algorithm 6) and
 * *value = sum of the excesses at height 0.  Requires a prior mf_maxflow.
 * On return, as for mf_maxflow.
 * Errors: MF_ERR_INVALID (any update out of range, u == v, cap < 0; nothing
 * is applied), MF_ERR_OVERFLOW (an updated pair's c(u,v)+c(v,u) above
 * INT32_MAX; nothing is applied), MF_ERR_STATE, MF_ERR_NOT_CONVERGED,
 * MF_ERR_OUT_OF_MEMORY, MF_ERR_DEVICE. */
mf_status mf_apply_batch(mf_graph* g, const mf_update* upd, int64_t k, int64_t* value);

/* As mf_apply_batch, with the k updates already in DEVICE memory on the
 * handle's device (for example a torch tensor of shape [k, 3], int32).  The
 * buffer is only read, on the handle's stream, before the call returns. */
mf_status mf_apply_batch_device(mf_graph* g, const mf_update* d_upd, int64_t k, int64_t* value);

/* Largest batch mf_apply_batch_device_noalloc takes. */
#define MF_NOALLOC_MAX_UPDATES 32768

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it):
 * mf_apply_batch_device without any allocation.  Same arguments, semantics
 * and result as mf_apply_batch_device; the updates are in device memory.
 * The batch scratch (the slot located for each update, the updates that
 * changed a capacity, the hash table of absent pairs) lives in one static
 * device array per GPU of about 1.8 MB, held by each GPU the library runs on
 * until the process ends; its hash table is cleared by every call.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (two
 * handles used from different threads or streams) race, and the caller must
 * order them.  Nothing else is allocated: the handle's own buffers come from
 * its first mf_maxflow, and no new HIP graph is instantiated (an iteration
 * captured by an earlier call is replayed, else the kernels are launched one
 * by one).
 * Errors: MF_ERR_INVALID (as mf_apply_batch_device, or k above
 * MF_NOALLOC_MAX_UPDATES), MF_ERR_OVERFLOW, MF_ERR_STATE (no prior solve),
 * MF_ERR_OUT_OF_MEMORY (the batch inserts more pairs than the rows' free
 * slots hold: nothing is applied; mf_apply_batch_device re-lays the rows),
 * MF_ERR_NOT_CONVERGED, MF_ERR_DEVICE. */
mf_status mf_apply_batch_device_noalloc(mf_graph* g, const mf_update* d_upd, int64_t k, int64_t* value);

/* The minimum cut certified by the last solve (Sections 3.1 and 4.3):
 * source side A = {v : h(v) = |V|} under a global relabel of the final
 * residual graph, the vertices that cannot reach t or a deficient vertex in
 * it (when the solve ended after a round rather than a relabel, this call
 * runs that relabel first).  source_side: uint8[n] host buffer (1 = A,
 * 0 = B) or NULL; *cut_capacity = sum of c(u,v) over u in A, v in B, which
 * equals the last returned value.  Requires a prior solve.
 * Errors: MF_ERR_INVALID, MF_ERR_STATE, MF_ERR_DEVICE. */
mf_status mf_min_cut(mf_graph* g, uint8_t* source_side, int64_t* cut_capacity);

/* A maximum flow for the current capacities (Section 3.1's construction from
 * residuals, after completing the preflow: excess left on the source side is
 * returned to s and deficits on the sink side are filled from t, along
 * residual paths inside each side, Sections 3.1 and 4.3).  One entry per
 * merged directed pair with capacity > 0, sorted by (u, v): src[i], dst[i],
 * flow[i] with 0 <= flow <= c.  With all three arrays NULL only *count is
 * written (the number of entries).  Otherwise *count must hold the arrays'
 * length on input (MF_ERR_INVALID if it is too short) and receives the
 * number written.  The completion runs on a copy: the retained solver state
 * is not changed.
 * Errors: MF_ERR_INVALID, MF_ERR_STATE, MF_ERR_NOT_CONVERGED, MF_ERR_DEVICE. */
mf_status mf_get_flow(mf_graph* g, int64_t* count, int32_t* src, int32_t* dst, int32_t* flow);

/* The current capacities: one entry per directed pair with capacity > 0,
 * sorted by (u, v) (the graph as mf_graph_load would take it back).  With all
 * three arrays NULL only *count is written; otherwise *count holds the
 * arrays' length on input (MF_ERR_INVALID if too short) and receives the
 * number written.  Does not change the solver state. */
mf_status mf_get_edges(mf_graph* g, int64_t* count, int32_t* src, int32_t* dst, int32_t* cap);

/* Move the graph's retained state (the Bi-CSR with its residuals and
 * capacities, excesses and heights) from device memory into pinned host
 * memory owned by the handle, and free the device memory it held (a few
 * hundred bytes of counters stay).  While offloaded every call except
 * mf_graph_restore, mf_get_stats and mf_graph_free returns MF_ERR_STATE.  The
 * host buffers are kept for the next offload and released by mf_graph_free.
 * For callers that keep more graphs than fit in HBM: a restored graph
 * resumes exactly where it was (Section 4's repair needs the retained state).
 * Errors: MF_ERR_INVALID, MF_ERR_STATE (already offloaded),
 * MF_ERR_OUT_OF_MEMORY (host buffers; nothing changed), MF_ERR_DEVICE. */
mf_status mf_graph_offload(mf_graph* g);

/* Re-allocate device memory and copy the offloaded state back.  Errors:
 * MF_ERR_INVALID, MF_ERR_STATE (not offloaded), MF_ERR_OUT_OF_MEMORY (device
 * memory; the graph stays offloaded, nothing lost), MF_ERR_DEVICE. */
mf_status mf_graph_restore(mf_graph* g);

/* Apply the tuning fields of *opt (kernel_cycles, bfs_alpha, bfs_beta,
 * round_div, bin_thread_max, bin_wave_max, long_row_cycles), its loop and
 * relabel settings (bfs_first_chunk ... trace) and max_iterations to a live
 * handle, for autotuners that time one handle under several settings; other
 * fields are ignored and every field left 0 takes its default.  Results never
 * depend on them (max_iterations only decides MF_ERR_NOT_CONVERGED).
 * Errors: MF_ERR_INVALID (NULL, struct_size, bin_wave_max below
 * bin_thread_max, bfs_bottom_up outside 0..2), MF_ERR_STATE (offloaded). */
mf_status mf_graph_tune(mf_graph* g, const mf_options* opt);

/* Counters and sizes; see mf_stats (device_bytes is the counters' size while
 * offloaded). */
mf_status mf_get_stats(const mf_graph* g, mf_stats* out);

/* Per-kernel event timing.  class_mask selects kernel classes by bit (bit c =
 * index c of mf_stats.kernel_ms; 0 turns timing off, 0xFF times every class)
 * and clears the totals.  Each launch of a selected class is bracketed by HIP
 * events on the handle's stream; mf_stats accumulates their durations, the
 * launch counts and the algorithmic bytes of the selected classes. */
mf_status mf_profile(mf_graph* g, int32_t class_mask);

/* Diagnostic: reset to zero flow, saturate the source, run one global
 * relabel (Algorithm 4) and one worklist build (Section 5.2), and copy out
 * heights int32[n], excesses int64[n] and the active vertices (any order,
 * *n_active of them; buffer of n entries).  Any output may be NULL.  Leaves
 * the handle needing a new mf_maxflow before repairs. */
mf_status mf_debug_initial_labels(mf_graph* g, int32_t* heights, int64_t* excess,
                                  int32_t* active, int32_t* n_active);

/* Diagnostic: one round of the loop on the current heights, as a solve runs
 * it between global relabels: the active-vertex worklist (Section 5.2), then
 * with parts bit 0 the push-relabel kernel over it (Algorithm 2) and with bit 1
 * the remove-invalid-edges kernel over the same rows (Algorithm 3).  For
 * checking the invariants between kernels (mf_debug_check_invariants), for
 * example after mf_debug_initial_labels.  Afterwards the handle needs a new
 * mf_maxflow before repairs, cuts and flows (its heights are no longer a
 * terminating relabel's).
 * Errors: MF_ERR_INVALID (parts outside 0..3), MF_ERR_STATE (offloaded),
 * MF_ERR_DEVICE. */
mf_status mf_debug_round(mf_graph* g, int32_t parts);

/* Diagnostic: check on the device what Section 3.1 states for the residual
 * state between kernels, over every used slot and vertex.  counts: int64[8]
 * host buffer receiving
 *   [0] slots with a negative residual (c_f >= 0 must hold)
 *   [1] slots whose pair's two residuals do not sum to its two capacities
 *   [2] slots whose pairing is broken (rev[rev[j]] != j, the reverse slot's
 *       column is not the row's vertex, or capsum != cap + cap of the reverse)
 *   [3] vertices whose excess differs from their net inflow, the sum over
 *       their row of (c_f - c)
 *   [4] the sum of all excesses (0 when no flow is lost or created)
 *   [5] vertices with a height outside [0, |V|]
 *   [6] residual slots u->v with h(u) < |V| and h(u) > h(v) + 1 (none after a
 *       fresh relabel or a remove-invalid-edges round)
 *   [7] active vertices (outside {s, t}, e > 0, h < |V|; none when a solve ends)
 * Does not change the state.  Errors: MF_ERR_INVALID, MF_ERR_STATE
 * (offloaded), MF_ERR_DEVICE. */
mf_status mf_debug_check_invariants(mf_graph* g, int64_t* counts);

/* Diagnostic: run the device self-test of the wave primitives the kernels
 * rely on (64-lane DPP minimum, wave prefix sum) on `device` (-1: current)
 * and compare each result with a lane-by-lane loop.  MF_OK when all agree,
 * MF_ERR_DEVICE otherwise. */
mf_status mf_debug_selftest(int32_t device);

/* Diagnostic: atomic throughput on `device` (-1: current): n atomicAdds of
 * `width` bytes (4 or 8) spread over n distinct addresses in a scattered
 * order (n below 2^31), timed with HIP events after one warm-up
 * launch; *ops_per_s receives the rate.  The reference point for the push and
 * relabel kernels, whose updates are scattered atomics.  Errors:
 * MF_ERR_INVALID, MF_ERR_DEVICE. */
mf_status mf_debug_atomic_probe(int32_t device, int64_t n, int32_t width, double* ops_per_s);

/* Release the handle and its device memory.  NULL is ignored. */
void mf_graph_free(mf_graph* g);

/* ---- many independent graphs in one launch --------------------------------
 * A batch holds num_graphs graphs in pooled device memory.  mf_batch_maxflow
 * solves all of them from zero flow in one launch (one workgroup per graph
 * runs the whole loop of Algorithm 1, largest graphs first);
 * mf_batch_apply repairs all of them after their update batches (Algorithm
 * 5) in two launches.  Each graph's value is exactly what mf_maxflow /
 * mf_apply_batch return for it alone. */
typedef struct mf_batch mf_batch;

/* num_graphs >= 1 graphs, graph i with n[i] vertices, edges
 * [edge_offset[i], edge_offset[i+1]) of the concatenated host arrays src,
 * dst, cap (vertex ids local to the graph, 0..n[i]-1), source s[i], sink
 * t[i].  edge_offset has num_graphs + 1 entries, edge_offset[0] = 0.  Every
 * graph is validated as in mf_graph_load before anything is allocated.
 * opt (NULL: defaults) applies to every graph.  On success *out owns the
 * pooled device memory until mf_batch_free.  Errors: MF_ERR_INVALID (a null
 * array, offsets that do not start at 0 or decrease, an invalid graph or
 * options), MF_ERR_OVERFLOW (a capacity pair above INT32_MAX, or the pool's
 * slots or vertices above INT32_MAX),
 * MF_ERR_OUT_OF_MEMORY, MF_ERR_DEVICE; *out is not written on error. */
mf_status mf_batch_load(int32_t num_graphs, const int32_t* n, const int64_t* edge_offset,
                        const int32_t* src, const int32_t* dst, const int32_t* cap, const int32_t* s,
                        const int32_t* t, const mf_options* opt, mf_batch** out);

/* Max-flow value of every graph from zero flow; values: int64[num_graphs].
 * MF_ERR_NOT_CONVERGED if any graph hit the iteration cap (the other values
 * are still written). */
mf_status mf_batch_maxflow(mf_batch* b, int64_t* values);

/* Apply graph i's updates upd[update_offset[i] .. update_offset[i+1]) (host
 * memory, ids local to the graph, same semantics as mf_apply_batch) to every
 * graph and return every new value.  All updates of all graphs are validated
 * first; on MF_ERR_INVALID or MF_ERR_OVERFLOW (a capacity pair above
 * INT32_MAX, or a row whose insertion slack would be exceeded: load with more
 * slack) no graph is changed.  Requires a prior mf_batch_maxflow. */
mf_status mf_batch_apply(mf_batch* b, const int64_t* update_offset, const mf_update* upd,
                         int64_t* values);

/* Loop iterations (global relabels) of each graph in the last call
 * (int32[num_graphs], or NULL) and the call's host wall time in ms (or
 * NULL).  Errors: MF_ERR_INVALID (b NULL). */
mf_status mf_batch_info(const mf_batch* b, int32_t* iterations, double* last_ms);

/* mf_graph_tune for a batch: the same fields plus batch_block (threads per
 * graph: 256, 512 or 1024).  Errors: MF_ERR_INVALID, MF_ERR_DEVICE. */
mf_status mf_batch_tune(mf_batch* b, const mf_options* opt);

/* Profiling of the batched solve: with on != 0 every later mf_batch_maxflow
 * and mf_batch_apply times its solve launch (the one that runs every graph's
 * loop) with HIP events on the batch's stream and counts the algorithmic
 * bytes its kernels move on the device (Bi-CSR slots and vertex words
 * visited, as mf_stats.kernel_bytes counts them for one graph); on == 0
 * turns it off.  Errors: MF_ERR_INVALID, MF_ERR_DEVICE. */
mf_status mf_batch_profile(mf_batch* b, int32_t on);

/* The last profiled call's solve launch: its event time in ms and the
 * algorithmic bytes its kernels moved (0 when not profiling); either output
 * may be NULL.  Errors: MF_ERR_INVALID (b NULL). */
mf_status mf_batch_kernel_stats(const mf_batch* b, double* kernel_ms, double* alg_bytes);

void mf_batch_free(mf_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
