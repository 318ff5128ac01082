"""Seeded generators: determinism, shapes, and update-mix bookkeeping."""
import numpy as np
import pytest

from paper_2511_01235_amd import gen


def _model(g):
    d = {}
    for a, b, x in zip(g.src.tolist(), g.dst.tolist(), g.cap.tolist()):
        d[(a, b)] = d.get((a, b), 0) + x
    return d


def test_er_shape_and_determinism():
    g1 = gen.erdos_renyi(2000, 16000, 100, seed=11)
    g2 = gen.erdos_renyi(2000, 16000, 100, seed=11)
    assert g1.m == 16000 and g1.s == 0 and g1.t == 1999
    assert np.array_equal(g1.src, g2.src) and np.array_equal(g1.cap, g2.cap)
    key = g1.src.astype(np.int64) * 2000 + g1.dst
    assert np.unique(key).size == 16000 and (g1.src != g1.dst).all()
    assert g1.cap.min() >= 1 and g1.cap.max() <= 100


def test_grid_shape():
    g = gen.grid(16, 100, seed=3)
    assert g.n == 16 * 16 + 2 and g.m == 4 * 16 * 15 + 2 * 16
    assert (g.cap[g.src == g.s] == 1000).all() and (g.cap[g.dst == g.t] == 1000).all()


def test_rmat_source_sink_rule():
    g = gen.rmat(12, 16, 1000, seed=5)
    assert (g.src != g.dst).all()
    key = np.unique(g.src.astype(np.int64) * g.n + g.dst)
    outdeg = np.bincount(key // g.n, minlength=g.n)
    indeg = np.bincount(key % g.n, minlength=g.n)
    assert outdeg[g.s] == outdeg.max() and g.t != g.s
    indeg[g.s] = -1
    assert indeg[g.t] == indeg.max()


def test_batch_mix_and_state_tracking():
    for name in ("er2000", "rmat12", "grid64"):
        g, stream, k, nb = gen.workload(name)
        model = _model(g)
        for _ in range(3):
            before = dict(model)
            u, v, c = stream.next_batch(k)
            assert u.size == k and (u != v).all() and (c >= 0).all()
            keys = list(zip(u.tolist(), v.tolist()))
            assert len(set(keys)) == k  # generated batches hold distinct pairs
            old = np.array([before.get(p, 0) for p in keys])
            n_inc = int(((old > 0) & (c > old)).sum())
            n_dec = int(((old > 0) & (c < old)).sum())
            n_new = int((old == 0).sum())
            assert n_inc == round(0.4 * k) and n_dec == round(0.4 * k) and n_new == k - n_inc - n_dec
            for p, x in zip(keys, c.tolist()):
                model[p] = x
            cs, cd, cc = stream.current_edges()
            live = {p: x for p, x in model.items() if x > 0}
            assert live == dict(zip(zip(cs.tolist(), cd.tolist()), cc.tolist()))


def test_grid_patch_batches_stay_in_patch():
    g, stream, k, nb = gen.workload("grid256")
    u, v, c = stream.next_batch(k)
    W = 256
    rows = np.concatenate([u // W, v // W])
    cols = np.concatenate([u % W, v % W])
    assert rows.max() - rows.min() < 64 and cols.max() - cols.min() < 64


@pytest.mark.parametrize("kind", ["inc", "dec", "mixed"])
def test_paper_batch_shapes(kind):
    """Section 6.2's update files: existing edges only, distinct, direction of
    the change as requested, source/sink edges favoured, caps tracked."""
    g, st, _, _ = gen.workload("er2000")
    before = dict(zip(st.keys.tolist(), st.caps.tolist()))
    u, v, c = st.paper_batch(400, kind, st_bias=50.0)
    keys = u.astype(np.int64) * g.n + v
    assert np.unique(keys).size == keys.size
    old = np.array([before[k] for k in keys.tolist()])
    assert (old > 0).all()
    if kind == "inc":
        assert (c > old).all()
    elif kind == "dec":
        assert (c < old).all() and (c >= 0).all()
    else:
        assert ((c > old) | (c < old)).all() and (c > old).any() and (c < old).any()
    st_edges = np.mean((u == g.s) | (v == g.t))
    base = np.mean((g.src == g.s) | (g.dst == g.t))
    assert st_edges > 5 * base
    after = dict(zip(st.keys.tolist(), st.caps.tolist()))
    assert all(after[k] == x for k, x in zip(keys.tolist(), c.tolist()))
