"""Invariants of the seeded synthetic molecule generator (the stand-in for the
paper's PCQM4Mv2 / AISD HOMO-LUMO batches, Section 5.1 and Table 2)."""
import numpy as np
import pytest

from paper_2207_11333_amd import synth


@pytest.mark.parametrize("name", ["c0_small_fp32", "c1_train_fp32"])
def test_shapes_and_invariants(name):
    w = synth.WORKLOADS[name]
    b = w.batch()
    B, N, E = b.num_graphs, b.num_nodes, b.num_edges
    assert B == w.num_graphs
    assert b.x.shape == (N, 9) and b.x.dtype == np.float32
    assert b.edge_index.shape == (2, E) and b.edge_index.dtype == np.int32
    assert b.y.shape == (B,)
    sizes = np.diff(b.graph_ptr)
    assert sizes.min() >= w.n_lo and sizes.max() <= w.n_hi
    # one-hot atom type + 4 scalars
    assert np.all(b.x[:, :5].sum(1) == 1.0)
    src, dst = b.edge_index
    deg_in = np.bincount(dst, minlength=N)
    deg_out = np.bincount(src, minlength=N)
    assert deg_in.max() <= 4 and deg_in.min() >= 1
    assert np.array_equal(deg_in, deg_out)
    # both directions stored, consecutive, equal attributes
    assert np.array_equal(src[0::2], dst[1::2]) and np.array_equal(dst[0::2], src[1::2])
    if b.edge_attr is not None:
        assert np.array_equal(b.edge_attr[0::2], b.edge_attr[1::2])
        assert b.edge_attr.min() >= 0.9 and b.edge_attr.max() <= 1.6
    assert 2.0 <= E / N <= 2.3
    # connected (tree spans every graph), no self loops, no duplicate bonds
    assert np.all(src != dst)
    pairs = set(zip(src.tolist(), dst.tolist()))
    assert len(pairs) == E
    for g in range(B):
        lo, hi = b.graph_ptr[g], b.graph_ptr[g + 1]
        seen = {lo}
        stack = [lo]
        sel = (src >= lo) & (src < hi)
        adj = {}
        for s, d in zip(src[sel], dst[sel]):
            adj.setdefault(int(s), []).append(int(d))
        while stack:
            v = stack.pop()
            for u in adj.get(v, []):
                if u not in seen:
                    seen.add(u)
                    stack.append(u)
        assert len(seen) == hi - lo


def test_determinism_per_seed():
    a = synth.make_batch(7, 10, 5, 30, 1)
    b = synth.make_batch(7, 10, 5, 30, 1)
    c = synth.make_batch(8, 10, 5, 30, 1)
    for k in ("graph_ptr", "x", "edge_index", "edge_attr", "y"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert not np.array_equal(a.x.shape, c.x.shape) or not np.array_equal(a.x, c.x)


def test_params_packing_and_init():
    shape = synth.ModelShape(2, 8, 9, 1)
    p = synth.init_params(shape, 1)
    assert p.dtype == np.float32 and p.shape == (shape.num_params(),)
    offs = shape.offsets()
    off, shp = offs["l0.Wp"]
    W = p[off:off + np.prod(shp)]
    bound = np.sqrt(6.0 / (shp[0] + shp[1]))
    assert np.abs(W).max() <= bound and np.abs(W).max() > 0.8 * bound
    off, shp = offs["l1.bm"]
    assert np.abs(p[off:off + shp[0]]).max() <= 0.1
    assert np.array_equal(p, synth.init_params(shape, 1))


def test_select_and_concat_roundtrip():
    b = synth.make_batch(3, 5, 4, 9, 1)
    r = synth.select_graphs(b, range(5))
    for k in ("graph_ptr", "x", "edge_index", "edge_attr", "y"):
        assert np.array_equal(getattr(r, k), getattr(b, k))


def test_splitmix64_reference_values():
    """SplitMix64 from seed 0 (published test values of the generator as used
    to seed xoshiro/xorshift generators)."""
    got = synth.splitmix64_at(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                     0x06C45D188009454F]


def test_counter_init_bounds_and_moments():
    shape = synth.ModelShape(2, 32, 9, 1)
    p = synth.counter_init_params(shape.tensor_shapes(), 7)
    assert p.dtype == np.float32 and p.shape[0] == shape.num_params()
    for name, (off, shp) in shape.offsets().items():
        v = p[off:off + int(np.prod(shp))].astype(np.float64)
        a = np.sqrt(6.0 / (shp[0] + shp[1])) if len(shp) == 2 else 0.1
        assert np.all(np.abs(v) <= a * (1 + 1e-7)), name
        if v.size > 1000:
            # uniform on [-a, a): mean 0, variance a^2 / 3
            assert abs(v.mean()) < 0.05 * a and abs(v.var() / (a * a / 3) - 1) < 0.05, name
    assert not np.array_equal(p, synth.counter_init_params(shape.tensor_shapes(), 8))
