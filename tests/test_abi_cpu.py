"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/mf.h declares, and rejects invalid input before touching the
device (validation happens first, so these return without a GPU)."""
import os
import re

import numpy as np
import pytest

import paper_2511_01235_amd as mf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = mf.lib()
    names = _declared()
    assert "mf_graph_load" in names and "mf_apply_batch" in names and "mf_min_cut" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(mf.EXPORTED) == names


def test_status_strings():
    for code in range(7):
        assert mf.status_string(code)


@pytest.mark.parametrize("case", [
    dict(n=1, e=[[0, 0, 1]], s=0, t=0),
    dict(n=3, e=[[0, 1, 1]], s=1, t=1),
    dict(n=3, e=[[0, 1, 1]], s=-1, t=2),
    dict(n=3, e=[[0, 1, 1]], s=0, t=3),
    dict(n=3, e=[[0, 0, 1]], s=0, t=2),
    dict(n=3, e=[[0, 1, -1]], s=0, t=2),
    dict(n=3, e=[[0, 5, 1]], s=0, t=2),
    dict(n=3, e=[[-1, 1, 1]], s=0, t=2),
])
def test_load_rejects_invalid(case):
    e = np.array(case["e"], np.int64)
    with pytest.raises(mf.MFError) as ei:
        mf.mf_graph_load(case["n"], e[:, 0], e[:, 1], e[:, 2], case["s"], case["t"])
    assert ei.value.status == mf.MF_ERR_INVALID


def test_load_rejects_pair_overflow():
    big = 2**31 - 1
    for e in ([[0, 1, big], [0, 1, 1]], [[0, 1, big], [1, 0, 1]]):
        e = np.array(e, np.int64)
        with pytest.raises(mf.MFError) as ei:
            mf.mf_graph_load(3, e[:, 0], e[:, 1], e[:, 2], 0, 2)
        assert ei.value.status == mf.MF_ERR_OVERFLOW


def test_options_struct_size_checked():
    o = mf.mf_default_options()
    assert o.struct_size == mf.C.sizeof(mf.Options)
    o.struct_size = 7
    with pytest.raises(mf.MFError) as ei:
        mf.mf_graph_load(3, [0], [1], [1], 0, 2, o)
    assert ei.value.status == mf.MF_ERR_INVALID


def test_null_handle_calls():
    L = mf.lib()
    v = mf.C.c_int64()
    assert L.mf_maxflow(None, mf.C.byref(v)) == mf.MF_ERR_INVALID
    assert L.mf_apply_batch(None, None, 0, mf.C.byref(v)) == mf.MF_ERR_INVALID
    assert L.mf_min_cut(None, None, mf.C.byref(v)) == mf.MF_ERR_INVALID
    assert L.mf_get_stats(None, None) == mf.MF_ERR_INVALID
    L.mf_graph_free(None)


def test_batch_load_rejects_invalid():
    L = mf.lib()
    n = np.array([3, 3], np.int32)
    off = np.array([0, 1, 2], np.int64)
    src = np.array([0, 0], np.int32)
    dst = np.array([1, 1], np.int32)
    cap = np.array([1, -1], np.int32)  # negative capacity in graph 1
    s = np.array([0, 0], np.int32)
    t = np.array([2, 2], np.int32)
    h = mf.C.c_void_p()
    rc = L.mf_batch_load(2, n.ctypes.data, off.ctypes.data, src.ctypes.data, dst.ctypes.data,
                         cap.ctypes.data, s.ctypes.data, t.ctypes.data, None, mf.C.byref(h))
    assert rc == mf.MF_ERR_INVALID and not h.value
    assert L.mf_batch_maxflow(None, None) == mf.MF_ERR_INVALID
    L.mf_batch_free(None)


def test_half_an_allocator_is_rejected():
    """mf_options.alloc without .free (or the reverse) is refused before any
    device work, for graphs and batches."""
    import ctypes as C
    o = mf.mf_default_options()
    cb = mf.ALLOC_FN(lambda n, ctx: None)
    o.alloc = C.cast(cb, C.c_void_p).value
    src, dst, cap = (np.array([0], np.int32), np.array([1], np.int32), np.array([5], np.int32))
    with pytest.raises(mf.MFError) as ei:
        mf.mf_graph_load(3, src, dst, cap, 0, 2, o)
    assert ei.value.status == mf.MF_ERR_INVALID
    h = C.c_void_p()
    n = np.array([3], np.int32)
    off = np.array([0, 1], np.int64)
    s = np.array([0], np.int32)
    t = np.array([2], np.int32)
    st = mf.lib().mf_batch_load(1, n.ctypes.data, off.ctypes.data, src.ctypes.data, dst.ctypes.data,
                                cap.ctypes.data, s.ctypes.data, t.ctypes.data, C.byref(o), C.byref(h))
    assert st == mf.MF_ERR_INVALID and not h.value


def test_bad_tuning_is_rejected():
    o = mf.make_options(bin_thread_max=64, bin_wave_max=32)
    src, dst, cap = (np.array([0], np.int32), np.array([1], np.int32), np.array([5], np.int32))
    with pytest.raises(mf.MFError) as ei:
        mf.mf_graph_load(3, src, dst, cap, 0, 2, o)
    assert ei.value.status == mf.MF_ERR_INVALID
    with pytest.raises(mf.MFError):
        mf.mf_graph_load(3, src, dst, cap, 0, 2, mf.make_options(batch_block=300))


def test_loop_options_validated_before_the_device():
    """Loop and relabel settings travel in mf_options (no environment
    switches); an out-of-range variant is rejected before any device work."""
    o = mf.make_options(bfs_first_chunk=4, pipeline=-1, graph_capture=1, bfs_narrow_slots=-1)
    assert (o.bfs_first_chunk, o.pipeline, o.graph_capture, o.bfs_narrow_slots) == (4, -1, 1, -1)
    with pytest.raises(TypeError):
        mf.make_options(no_such_setting=1)
    bad = mf.make_options(bfs_bottom_up=3)
    with pytest.raises(mf.MFError) as ei:
        mf.mf_graph_load(3, [0], [1], [1], 0, 2, bad)
    assert ei.value.status == mf.MF_ERR_INVALID


def test_library_reads_no_environment_switches():
    """The product library takes every setting from mf_options: its sources
    call no getenv."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "paper_2511_01235_amd", "csrc", "*")):
        assert "getenv" not in open(path).read(), path


def _batch_load(n, off, e, s, t, opt=None):
    """mf_batch_load through the C ABI: returns (status, handle)."""
    import ctypes as C
    n = np.asarray(n, np.int32)
    off = np.asarray(off, np.int64)
    e = np.asarray(e, np.int32).reshape(-1, 3)
    src, dst, cap = (np.ascontiguousarray(e[:, i]) for i in range(3))
    s = np.asarray(s, np.int32)
    t = np.asarray(t, np.int32)
    h = C.c_void_p()
    rc = mf.lib().mf_batch_load(int(n.size), n.ctypes.data, off.ctypes.data, src.ctypes.data,
                                dst.ctypes.data, cap.ctypes.data, s.ctypes.data, t.ctypes.data,
                                C.byref(opt) if opt is not None else None, C.byref(h))
    return rc, h.value


@pytest.mark.parametrize("case,want", [
    (dict(n=[3], off=[1, 1], e=[[0, 1, 1]], s=[0], t=[2]), "invalid"),            # offsets start above 0
    (dict(n=[3, 3], off=[0, 1, 0], e=[[0, 1, 1]], s=[0, 0], t=[2, 2]), "invalid"),  # offsets decrease
    (dict(n=[3, 3], off=[0, 1, 2], e=[[0, 1, 1], [0, 1, 1]], s=[0, 1], t=[2, 1]), "invalid"),  # s == t
    (dict(n=[3, 3], off=[0, 1, 2], e=[[0, 1, 1], [0, 3, 1]], s=[0, 0], t=[2, 2]), "invalid"),  # vertex id
    (dict(n=[3], off=[0, 2], e=[[0, 1, 2**31 - 1], [1, 0, 1]], s=[0], t=[2]), "overflow"),  # pair sum
])
def test_batch_load_rejects_invalid(case, want):
    """The batched load validates every graph on the host before it touches the
    device: a bad offset table, an invalid graph or a capacity pair above int32
    is rejected and no handle is returned."""
    rc, h = _batch_load(**case)
    assert rc == {"invalid": mf.MF_ERR_INVALID, "overflow": mf.MF_ERR_OVERFLOW}[want]
    assert not h


def test_batch_load_rejects_bad_options():
    import ctypes as C
    opt = mf.make_options()
    opt.struct_size = C.sizeof(opt) - 4
    rc, h = _batch_load([3], [0, 1], [[0, 1, 1]], [0], [2], opt=opt)
    assert rc == mf.MF_ERR_INVALID and not h
    rc, h = _batch_load([], [0], np.zeros((0, 3)), [], [])
    assert rc == mf.MF_ERR_INVALID and not h

