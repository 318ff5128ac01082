"""MI355X-native dynamic max-flow: Python binding of the C ABI in include/mf.h.

Every function here only marshals arguments into the HIP library
`libmf.so` (built in-tree by `build.py`) and back; all computation runs in
that library's gfx950 kernels.  There is no fallback: if the library is not
built, or the device is unusable, the calls raise.

Names match the C ABI: mf_graph_load, mf_maxflow, mf_apply_batch,
mf_apply_batch_device, mf_min_cut, mf_get_flow, mf_get_stats, mf_profile,
mf_debug_initial_labels, mf_debug_selftest, mf_graph_free.  `MaxFlowGraph`
wraps a handle for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

MF_OK = 0
MF_ERR_INVALID = 1
MF_ERR_OUT_OF_MEMORY = 2
MF_ERR_OVERFLOW = 3
MF_ERR_DEVICE = 4
MF_ERR_NOT_CONVERGED = 5
MF_ERR_STATE = 6

# every symbol include/mf.h declares
EXPORTED = ["mf_default_options", "mf_status_string", "mf_graph_load", "mf_maxflow",
            "mf_apply_batch", "mf_apply_batch_device", "mf_apply_batch_device_noalloc", "mf_min_cut", "mf_get_flow", "mf_get_edges",
            "mf_graph_offload", "mf_graph_restore", "mf_graph_tune", "mf_get_stats", "mf_profile",
            "mf_debug_initial_labels", "mf_debug_selftest", "mf_debug_atomic_probe", "mf_debug_round",
            "mf_debug_check_invariants", "mf_graph_free", "mf_batch_load", "mf_batch_maxflow",
            "mf_batch_apply", "mf_batch_info", "mf_batch_tune", "mf_batch_profile", "mf_batch_kernel_stats",
            "mf_batch_free"]

KERNEL_CLASSES = ["global_relabel", "push_relabel", "remove_invalid", "worklist", "batch", "init",
                  "relabel_seed_narrow", "unused7"]


class MFError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("device", C.c_int32), ("stream", C.c_void_p),
                ("kernel_cycles", C.c_int32), ("topology_driven", C.c_int32),
                ("insert_slack_min", C.c_int32), ("insert_slack_pct", C.c_int32),
                ("max_iterations", C.c_int64), ("cold_start", C.c_int32), ("relabel_mode", C.c_int32),
                ("bfs_alpha", C.c_int32), ("bfs_beta", C.c_int32), ("round_div", C.c_int32),
                ("bin_thread_max", C.c_int32), ("bin_wave_max", C.c_int32), ("batch_block", C.c_int32),
                ("push_pull", C.c_int32), ("alloc", C.c_void_p), ("free", C.c_void_p),
                ("alloc_ctx", C.c_void_p), ("long_row_cycles", C.c_int32)] + \
        [(name, C.c_int32) for name in ("bfs_first_chunk", "bfs_narrow_slots", "bfs_medium_slots",
                                        "bfs_medium_blocks", "bfs_level_blocks", "bfs_bottom_up",
                                        "bfs_lds_bitmap", "bfs_stage_min", "round_min", "round_max",
                                        "round_scan", "queue_rounds", "pipeline", "graph_capture", "trace",
                                        "round_narrow", "bfs_cap")]

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """Device memory for a handle from torch's caching allocator (launch the
    handle on `stream`, e.g. torch.cuda.current_stream()).  Pass as
    allocator=...; keep the object alive as long as the handle (the handle
    classes do)."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device, self.stream = device, stream

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
            except Exception:
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = ALLOC_FN(_alloc)
        self.free_fn = FREE_FN(_free)

# loop and relabel settings of a single-graph handle (0 = default; switches 1 on, -1 off)
LOOP_FIELDS = ("bfs_first_chunk", "bfs_narrow_slots", "bfs_medium_slots", "bfs_medium_blocks",
               "bfs_level_blocks", "bfs_bottom_up", "bfs_lds_bitmap", "bfs_stage_min", "round_min",
               "round_max", "round_scan", "queue_rounds", "pipeline", "graph_capture", "trace", "round_narrow",
               "bfs_cap")
# fields mf_graph_tune / mf_batch_tune apply to a live handle (mf_graph_tune also the loop fields)
TUNING_FIELDS = ("kernel_cycles", "bfs_alpha", "bfs_beta", "round_div", "bin_thread_max", "bin_wave_max",
                 "batch_block", "long_row_cycles", "max_iterations") + LOOP_FIELDS


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("pairs", C.c_int64), ("slots", C.c_int64),
                ("slot_capacity", C.c_int64), ("device_bytes", C.c_int64),
                ("kernel_cycles", C.c_int32), ("relayouts", C.c_int32),
                ("last_iterations", C.c_int64), ("last_bfs_levels", C.c_int64),
                ("last_active_sum", C.c_int64), ("last_new_pairs", C.c_int64),
                ("last_ms", C.c_double), ("kernel_ms", C.c_double * 8),
                ("kernel_launches", C.c_int64 * 8), ("kernel_bytes", C.c_double * 8),
                ("last_rounds", C.c_int64), ("last_capped_relabels", C.c_int64)]


class Update(C.Structure):
    _fields_ = [("u", C.c_int32), ("v", C.c_int32), ("cap", C.c_int32)]


_lib = None


def lib():
    """Load libmf.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_2511_01235_amd.build` or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.mf_default_options.argtypes = [C.POINTER(Options)]
        L.mf_default_options.restype = None
        L.mf_status_string.argtypes = [C.c_int]
        L.mf_status_string.restype = C.c_char_p
        L.mf_graph_load.argtypes = [i32, i64, vp, vp, vp, i32, i32, C.POINTER(Options), C.POINTER(vp)]
        L.mf_maxflow.argtypes = [vp, C.POINTER(i64)]
        L.mf_apply_batch.argtypes = [vp, vp, i64, C.POINTER(i64)]
        L.mf_apply_batch_device.argtypes = [vp, vp, i64, C.POINTER(i64)]
        L.mf_apply_batch_device_noalloc.argtypes = [vp, vp, i64, C.POINTER(i64)]
        L.mf_min_cut.argtypes = [vp, vp, C.POINTER(i64)]
        L.mf_get_flow.argtypes = [vp, C.POINTER(i64), vp, vp, vp]
        L.mf_get_edges.argtypes = [vp, C.POINTER(i64), vp, vp, vp]
        L.mf_graph_offload.argtypes = [vp]
        L.mf_graph_tune.argtypes = [vp, C.POINTER(Options)]
        L.mf_batch_tune.argtypes = [vp, C.POINTER(Options)]
        L.mf_graph_restore.argtypes = [vp]
        L.mf_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.mf_profile.argtypes = [vp, i32]
        L.mf_debug_initial_labels.argtypes = [vp, vp, vp, vp, C.POINTER(i32)]
        L.mf_debug_selftest.argtypes = [i32]
        L.mf_debug_atomic_probe.argtypes = [i32, i64, i32, C.POINTER(C.c_double)]
        L.mf_debug_round.argtypes = [vp, i32]
        L.mf_debug_check_invariants.argtypes = [vp, vp]
        L.mf_graph_free.argtypes = [vp]
        L.mf_graph_free.restype = None
        L.mf_batch_load.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Options), C.POINTER(vp)]
        L.mf_batch_maxflow.argtypes = [vp, vp]
        L.mf_batch_apply.argtypes = [vp, vp, vp, vp]
        L.mf_batch_info.argtypes = [vp, vp, C.POINTER(C.c_double)]
        L.mf_batch_profile.argtypes = [vp, i32]
        L.mf_batch_kernel_stats.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mf_batch_free.argtypes = [vp]
        L.mf_batch_free.restype = None
        for name in ["mf_graph_load", "mf_maxflow", "mf_apply_batch", "mf_apply_batch_device",
                     "mf_apply_batch_device_noalloc",
                     "mf_min_cut", "mf_get_flow", "mf_get_edges", "mf_graph_offload", "mf_graph_restore",
                     "mf_graph_tune", "mf_batch_tune",
                     "mf_get_stats", "mf_profile",
                     "mf_debug_initial_labels", "mf_debug_selftest", "mf_debug_atomic_probe", "mf_debug_round",
                     "mf_debug_check_invariants", "mf_batch_load",
                     "mf_batch_maxflow", "mf_batch_apply", "mf_batch_info", "mf_batch_profile",
                     "mf_batch_kernel_stats"]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().mf_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != MF_OK:
        raise MFError(status, where)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def mf_default_options() -> Options:
    o = Options()
    lib().mf_default_options(C.byref(o))
    return o


def make_options(kernel_cycles=0, topology_driven=False, insert_slack_min=0, insert_slack_pct=0,
                 max_iterations=0, stream=None, device=-1, warm_start=True,
                 relabel_mode=0, bfs_alpha=0, bfs_beta=0, round_div=0, bin_thread_max=0, bin_wave_max=0,
                 batch_block=0, push_pull=False, allocator=None, long_row_cycles=0, **loop) -> Options:
    """Options for a handle; `loop` takes any of LOOP_FIELDS."""
    bad = set(loop) - set(LOOP_FIELDS)
    if bad:
        raise TypeError(f"unknown options: {sorted(bad)}")
    o = mf_default_options()
    for name, val in loop.items():
        setattr(o, name, int(val))
    o.push_pull = int(bool(push_pull))
    if allocator is not None:
        o.alloc = C.cast(allocator.alloc_fn, C.c_void_p).value
        o.free = C.cast(allocator.free_fn, C.c_void_p).value
    o.bfs_alpha, o.bfs_beta, o.round_div = int(bfs_alpha), int(bfs_beta), int(round_div)
    o.bin_thread_max, o.bin_wave_max, o.batch_block = int(bin_thread_max), int(bin_wave_max), int(batch_block)
    o.long_row_cycles = int(long_row_cycles)
    o.cold_start = 0 if warm_start else 1
    o.relabel_mode = int(relabel_mode)
    o.kernel_cycles = kernel_cycles
    o.topology_driven = int(bool(topology_driven))
    o.insert_slack_min = insert_slack_min
    o.insert_slack_pct = insert_slack_pct
    o.max_iterations = max_iterations
    o.device = device
    if stream is not None:
        o.stream = stream if isinstance(stream, int) else int(stream.cuda_stream)
    return o


def mf_graph_load(n, src, dst, cap, s, t, opt: Options | None = None) -> int:
    src, dst, cap = _i32(src), _i32(dst), _i32(cap)
    if not (src.size == dst.size == cap.size):
        raise ValueError("src, dst and cap must have the same length")
    h = C.c_void_p()
    st = lib().mf_graph_load(int(n), int(src.size), src.ctypes.data, dst.ctypes.data,
                             cap.ctypes.data, int(s), int(t),
                             C.byref(opt) if opt is not None else None, C.byref(h))
    _check(st, "mf_graph_load")
    return h.value


def mf_maxflow(g) -> int:
    v = C.c_int64()
    _check(lib().mf_maxflow(g, C.byref(v)), "mf_maxflow")
    return v.value


def _updates_host(u, v=None, c=None):
    if v is None:
        arr = np.ascontiguousarray(u, dtype=np.int32).reshape(-1, 3)
    else:
        arr = np.ascontiguousarray(np.stack([_i32(u), _i32(v), _i32(c)], axis=1))
    return arr


def mf_apply_batch(g, u, v=None, c=None) -> int:
    """Updates from host memory: (u, v, c) arrays, or one [k, 3] int32 array."""
    arr = _updates_host(u, v, c)
    val = C.c_int64()
    _check(lib().mf_apply_batch(g, arr.ctypes.data, arr.shape[0], C.byref(val)), "mf_apply_batch")
    return val.value


def mf_apply_batch_device(g, updates) -> int:
    """Updates already on the device: a contiguous int32 torch tensor [k, 3]."""
    if updates.dtype.__str__() != "torch.int32" or not updates.is_contiguous() or updates.dim() != 2 \
            or updates.shape[1] != 3 or not updates.is_cuda:
        raise ValueError("expected a contiguous int32 cuda tensor of shape [k, 3]")
    val = C.c_int64()
    _check(lib().mf_apply_batch_device(g, updates.data_ptr(), updates.shape[0], C.byref(val)),
           "mf_apply_batch_device")
    return val.value


NOALLOC_MAX_UPDATES = 32768


def mf_apply_batch_device_noalloc(g, updates) -> int:
    """As mf_apply_batch_device, allocating nothing (batch scratch in the GPU's
    static array; at most NOALLOC_MAX_UPDATES updates)."""
    if updates.dtype.__str__() != "torch.int32" or not updates.is_contiguous() or updates.dim() != 2 \
            or updates.shape[1] != 3 or not updates.is_cuda:
        raise ValueError("expected a contiguous int32 cuda tensor of shape [k, 3]")
    val = C.c_int64()
    _check(lib().mf_apply_batch_device_noalloc(g, updates.data_ptr(), updates.shape[0], C.byref(val)),
           "mf_apply_batch_device_noalloc")
    return val.value


def mf_min_cut(g, n: int):
    side = np.zeros(n, np.uint8)
    c = C.c_int64()
    _check(lib().mf_min_cut(g, side.ctypes.data, C.byref(c)), "mf_min_cut")
    return side, c.value


def mf_get_flow(g):
    cnt = C.c_int64()
    _check(lib().mf_get_flow(g, C.byref(cnt), None, None, None), "mf_get_flow")
    k = cnt.value
    cnt = C.c_int64(k)
    src = np.zeros(k, np.int32)
    dst = np.zeros(k, np.int32)
    flow = np.zeros(k, np.int32)
    _check(lib().mf_get_flow(g, C.byref(cnt), src.ctypes.data, dst.ctypes.data, flow.ctypes.data),
           "mf_get_flow")
    k = cnt.value
    return src[:k], dst[:k], flow[:k]


def mf_get_edges(g):
    """Current (src, dst, cap) of every pair with capacity > 0, sorted by (u, v)."""
    cnt = C.c_int64()
    _check(lib().mf_get_edges(g, C.byref(cnt), None, None, None), "mf_get_edges")
    k = cnt.value
    src, dst, cap = np.zeros(k, np.int32), np.zeros(k, np.int32), np.zeros(k, np.int32)
    cnt = C.c_int64(k)
    _check(lib().mf_get_edges(g, C.byref(cnt), src.ctypes.data, dst.ctypes.data, cap.ctypes.data),
           "mf_get_edges")
    k = cnt.value
    return src[:k], dst[:k], cap[:k]


def mf_graph_tune(g, **tuning):
    """Apply tuning fields (see TUNING_FIELDS; 0 = default) to a live handle."""
    bad = set(tuning) - set(TUNING_FIELDS)
    if bad:
        raise TypeError(f"not tuning fields: {sorted(bad)}")
    _check(lib().mf_graph_tune(g, C.byref(make_options(**tuning))), "mf_graph_tune")


def mf_graph_offload(g):
    _check(lib().mf_graph_offload(g), "mf_graph_offload")


def mf_graph_restore(g):
    _check(lib().mf_graph_restore(g), "mf_graph_restore")


def mf_get_stats(g) -> dict:
    s = Stats()
    _check(lib().mf_get_stats(g, C.byref(s)), "mf_get_stats")
    out = {name: getattr(s, name) for name, _ in Stats._fields_
           if name not in ("kernel_ms", "kernel_launches", "kernel_bytes")}
    out["kernel_ms"] = dict(zip(KERNEL_CLASSES, list(s.kernel_ms)))
    out["kernel_launches"] = dict(zip(KERNEL_CLASSES, list(s.kernel_launches)))
    out["kernel_bytes"] = dict(zip(KERNEL_CLASSES, list(s.kernel_bytes)))
    return out


def mf_profile(g, class_mask: int = 0xFF):
    """class_mask: bit c times kernel class KERNEL_CLASSES[c]; 0 turns timing off."""
    _check(lib().mf_profile(g, int(class_mask)), "mf_profile")


def mf_debug_initial_labels(g, n: int):
    h = np.zeros(n, np.int32)
    e = np.zeros(n, np.int64)
    act = np.zeros(n, np.int32)
    na = C.c_int32()
    _check(lib().mf_debug_initial_labels(g, h.ctypes.data, e.ctypes.data, act.ctypes.data,
                                         C.byref(na)), "mf_debug_initial_labels")
    return h, e, act[:na.value].copy()


def mf_debug_selftest(device: int = -1) -> int:
    return int(lib().mf_debug_selftest(int(device)))


def mf_debug_atomic_probe(n: int = 1 << 26, width: int = 4, device: int = -1) -> float:
    """Scattered atomicAdd throughput (ops/s) on n distinct addresses."""
    r = C.c_double()
    _check(lib().mf_debug_atomic_probe(int(device), int(n), int(width), C.byref(r)), "mf_debug_atomic_probe")
    return r.value


INVARIANT_NAMES = ("negative_residuals", "pair_sums", "pair_links", "excess_mismatches", "excess_total",
                   "heights_out_of_range", "steep_slots", "active")


def mf_debug_round(g, parts: int = 3):
    """parts bit 0: push-relabel round, bit 1: remove-invalid-edges round, over a fresh worklist."""
    _check(lib().mf_debug_round(g, int(parts)), "mf_debug_round")


def mf_debug_check_invariants(g) -> dict:
    out = np.zeros(8, np.int64)
    _check(lib().mf_debug_check_invariants(g, out.ctypes.data), "mf_debug_check_invariants")
    return dict(zip(INVARIANT_NAMES, out.tolist()))


def mf_graph_free(g):
    if g:
        lib().mf_graph_free(g)


class MaxFlowGraph:
    """Owns one mf_graph handle."""

    def __init__(self, n, src, dst, cap, s, t, **options):
        self.n, self.s, self.t = int(n), int(s), int(t)
        self._allocator = options.get("allocator")   # the callbacks must outlive the handle
        opt = make_options(**options) if options else None
        self.h = mf_graph_load(n, src, dst, cap, s, t, opt)

    def maxflow(self) -> int:
        return mf_maxflow(self.h)

    def apply_batch(self, u, v=None, c=None) -> int:
        return mf_apply_batch(self.h, u, v, c)

    def apply_batch_device(self, updates) -> int:
        return mf_apply_batch_device(self.h, updates)

    def apply_batch_device_noalloc(self, updates) -> int:
        return mf_apply_batch_device_noalloc(self.h, updates)

    def min_cut(self):
        return mf_min_cut(self.h, self.n)

    def get_flow(self):
        return mf_get_flow(self.h)

    def get_edges(self):
        return mf_get_edges(self.h)

    def tune(self, **tuning):
        mf_graph_tune(self.h, **tuning)

    def offload(self):
        mf_graph_offload(self.h)

    def restore(self):
        mf_graph_restore(self.h)

    def stats(self) -> dict:
        return mf_get_stats(self.h)

    def profile(self, class_mask=0xFF):
        mf_profile(self.h, class_mask)

    def initial_labels(self):
        return mf_debug_initial_labels(self.h, self.n)

    def debug_round(self, parts=3):
        mf_debug_round(self.h, parts)

    def invariants(self) -> dict:
        return mf_debug_check_invariants(self.h)

    def close(self):
        if self.h:
            mf_graph_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MaxFlowBatch:
    """Many independent graphs solved together (mf_batch_*).  graphs: a list of
    objects with n, src, dst, cap, s, t (for example gen.Graph)."""

    def __init__(self, graphs, **options):
        self.G = len(graphs)
        self._allocator = options.get("allocator")
        n = np.array([g.n for g in graphs], np.int32)
        off = np.zeros(self.G + 1, np.int64)
        off[1:] = np.cumsum([g.src.size for g in graphs])
        cat = lambda name: _i32(np.concatenate([getattr(g, name) for g in graphs]) if self.G else [])
        src, dst, cap = cat("src"), cat("dst"), cat("cap")
        s = np.array([g.s for g in graphs], np.int32)
        t = np.array([g.t for g in graphs], np.int32)
        opt = make_options(**options) if options else None
        h = C.c_void_p()
        _check(lib().mf_batch_load(self.G, n.ctypes.data, off.ctypes.data, src.ctypes.data,
                                   dst.ctypes.data, cap.ctypes.data, s.ctypes.data, t.ctypes.data,
                                   C.byref(opt) if opt is not None else None, C.byref(h)),
               "mf_batch_load")
        self.h = h.value

    def maxflow(self):
        vals = np.zeros(self.G, np.int64)
        _check(lib().mf_batch_maxflow(self.h, vals.ctypes.data), "mf_batch_maxflow")
        return vals

    def apply(self, batches):
        """batches: one (u, v, c) triple of arrays per graph."""
        off = np.zeros(self.G + 1, np.int64)
        off[1:] = np.cumsum([np.asarray(b[0]).size for b in batches])
        upd = np.zeros((int(off[-1]), 3), np.int32)
        for i, (u, v, c) in enumerate(batches):
            upd[off[i]:off[i + 1], 0] = u
            upd[off[i]:off[i + 1], 1] = v
            upd[off[i]:off[i + 1], 2] = c
        vals = np.zeros(self.G, np.int64)
        _check(lib().mf_batch_apply(self.h, off.ctypes.data, upd.ctypes.data, vals.ctypes.data),
               "mf_batch_apply")
        return vals

    def tune(self, **tuning):
        bad = set(tuning) - set(TUNING_FIELDS)
        if bad:
            raise TypeError(f"not tuning fields: {sorted(bad)}")
        _check(lib().mf_batch_tune(self.h, C.byref(make_options(**tuning))), "mf_batch_tune")

    def profile(self, on=True):
        """Time each call's solve launch and count its algorithmic bytes."""
        _check(lib().mf_batch_profile(self.h, int(bool(on))), "mf_batch_profile")

    def kernel_stats(self):
        """(ms, algorithmic bytes) of the last profiled call's solve launch."""
        ms, nb = C.c_double(), C.c_double()
        _check(lib().mf_batch_kernel_stats(self.h, C.byref(ms), C.byref(nb)), "mf_batch_kernel_stats")
        return ms.value, nb.value

    def info(self):
        it = np.zeros(self.G, np.int32)
        ms = C.c_double()
        _check(lib().mf_batch_info(self.h, it.ctypes.data, C.byref(ms)), "mf_batch_info")
        return it, ms.value

    def close(self):
        if self.h:
            lib().mf_batch_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
