"""Pins of the GraphSAGE / CGCNN oracle (oracle/gclayers.py) against values
fixed by hand and by the mathematics: worked examples, a closed form, node
and edge permutation invariances, and central finite differences of the
hand-written adjoints."""
import math

import numpy as np
import pytest

from oracle import gclayers as gcl
from oracle import multitask as mt
from paper_2207_11333_amd import synth


def _batch(gp, x, ei, ea=None, y=None):
    x = np.asarray(x, np.float32)
    B = len(gp) - 1
    return synth.Batch(np.asarray(gp, np.int32), x, np.asarray(ei, np.int32).reshape(2, -1),
                       None if ea is None else np.asarray(ea, np.float32),
                       np.zeros(B, np.float32) if y is None else np.asarray(y, np.float32))


def _pack(parts, H, Tg=1):
    """Layer tensors, then Tg zero heads."""
    heads = [np.zeros(mt.head_size(H)) for _ in range(Tg)]
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts] + heads)


def test_sage_worked_example():
    """Three nodes, edges 0->1, 2->1, 1->0; node 2 has no in-edge.  With
    W_self = I, W_nbr = diag(2, -1), b = (0.5, 0):
      M = [x1, (x0 + x2)/2, 0] = [(3,-1), (0.5,3), (0,0)]
      u = x + W_nbr M + b = [(7.5,3), (4.5,-4), (0.5,4)], h' = ReLU(u)."""
    b = _batch([0, 3], [[1, 2], [3, -1], [0, 4]], [[0, 2, 1], [1, 1, 0]])
    W = np.array([[1, 0, 2, 0], [0, 1, 0, -1]], np.float64)
    params = _pack([W, [0.5, 0.0]], 2)
    rec = gcl.forward(params, b, gcl.SAGE, 1, 2)
    np.testing.assert_allclose(rec.layers[0].M, [[3, -1], [0.5, 3], [0, 0]])
    np.testing.assert_allclose(rec.layers[0].h_out, [[7.5, 3], [4.5, 0], [0.5, 4]])


def test_cgcnn_worked_example():
    """One edge 0->1, H = F0 = Fe = 1, identity embedding.  The filter reads the
    destination, the core the source: f = h_1 + w_e e, s = h_0.  With h_0 =
    ln(e - 1), softplus(s) = 1 exactly, so h'_1 = ReLU(h_1 + sigmoid(f)) and the
    source node (no in-edge) keeps ReLU(h_0)."""
    x0 = math.log(math.e - 1.0)
    for x1, we, e, want in [(0.0, 0.0, 5.0, 0.5),
                            (0.0, 1.0, 2.0, 1.0 / (1.0 + math.exp(-2.0))),
                            (-0.25, 0.5, 1.0, -0.25 + 1.0 / (1.0 + math.exp(-0.25)))]:
        b = _batch([0, 2], [[x0], [x1]], [[0], [1]], [[e]])
        params = _pack([[[1.0]], [0.0], [[1.0, 0.0, we], [0.0, 1.0, 0.0]], [0.0, 0.0]], 1)
        rec = gcl.forward(params, b, gcl.CGCNN, 1, 1)
        assert rec.layers[0].h_out[1, 0] == pytest.approx(max(want, 0.0), rel=1e-6)
        assert rec.layers[0].h_out[0, 0] == pytest.approx(x0, rel=1e-6)


def test_cgcnn_zero_weights_closed_form():
    """W = 0, b = 0: every message is sigmoid(0) softplus(0) = ln(2)/2, so
    h' = ReLU(h^0 + deg ln(2)/2) per feature, whatever the graph."""
    bt = synth.make_batch(5, 6, 3, 12, 1)
    H, L = 8, 2
    rng = np.random.default_rng(0)
    Wemb = rng.normal(size=(H, 9))
    bemb = rng.normal(size=H)
    zero_layers = []
    for _ in range(L):
        zero_layers += [np.zeros((2 * H, 2 * H + 1)), np.zeros(2 * H)]
    params = _pack([Wemb, bemb] + zero_layers, H)
    rec = gcl.forward(params, bt, gcl.CGCNN, L, H)
    deg = np.bincount(bt.edge_index[1], minlength=bt.num_nodes)[:, None]
    h = np.asarray(bt.x, np.float64) @ Wemb.T + bemb
    for l in range(L):
        h = np.maximum(h + deg * math.log(2.0) / 2.0, 0.0)
        np.testing.assert_allclose(rec.layers[l].h_out, h, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", gcl.KINDS)
def test_node_permutation_equivariance_and_edge_order(kind):
    bt = synth.make_batch(11, 5, 4, 14, 1)
    H, L = 8, 2
    params = synth.init_gc_params(kind, L, H, 7)
    rec = gcl.forward(params, bt, kind, L, H)
    rng = np.random.default_rng(3)
    # shuffle the COO edge list: nothing changes
    perm_e = rng.permutation(bt.num_edges)
    be = synth.Batch(bt.graph_ptr, bt.x, bt.edge_index[:, perm_e], bt.edge_attr[perm_e], bt.y)
    rec_e = gcl.forward(params, be, kind, L, H)
    np.testing.assert_allclose(rec_e.layers[-1].h_out, rec.layers[-1].h_out, rtol=1e-12)
    # relabel the nodes inside each graph: node outputs permute, predictions stay
    gp = bt.graph_ptr
    pi = np.concatenate([gp[b] + rng.permutation(gp[b + 1] - gp[b])
                         for b in range(bt.num_graphs)])      # new position -> old node
    inv = np.empty_like(pi)
    inv[pi] = np.arange(pi.size)
    bp = synth.Batch(gp, bt.x[pi], inv[bt.edge_index].astype(np.int32), bt.edge_attr, bt.y)
    rec_p = gcl.forward(params, bp, kind, L, H)
    np.testing.assert_allclose(rec_p.layers[-1].h_out, rec.layers[-1].h_out[pi],
                               rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(rec_p.y, rec.y, rtol=1e-11)


def _loss(params, bt, kind, L, H, Tg, Tn, yn):
    return gcl.forward(params, bt, kind, L, H, Tg, Tn, None, [0.7] * Tn, yn).loss


@pytest.mark.parametrize("kind,Tg,Tn", [("sage", 1, 0), ("cgcnn", 1, 0), ("sage", 2, 1),
                                        ("cgcnn", 1, 2)])
def test_gradients_central_differences(kind, Tg, Tn):
    """The hand-written adjoint against central differences of the loss, for
    every parameter of a tiny model (2 layers, H = 4, one edge feature)."""
    bt = synth.make_batch(21, 3, 3, 6, 1)
    H, L = 4, 2
    rng = np.random.default_rng(8)
    y = rng.normal(5.0, 1.0, size=(bt.num_graphs, Tg))
    bt = synth.Batch(bt.graph_ptr, bt.x, bt.edge_index, bt.edge_attr, y.astype(np.float32))
    yn = rng.normal(size=(bt.num_nodes, Tn)) if Tn else None
    params = synth.init_gc_params(kind, L, H, 31, graph_heads=Tg, node_heads=Tn)
    params = params.astype(np.float64)
    rec = gcl.forward(params, bt, kind, L, H, Tg, Tn, None, [0.7] * Tn, yn)
    grad, stats = gcl.backward(rec)
    assert grad.shape == params.shape
    h = 1e-6
    worst = 0.0
    for j in range(params.shape[0]):
        p1, p2 = params.copy(), params.copy()
        p1[j] += h
        p2[j] -= h
        fd = (_loss(p1, bt, kind, L, H, Tg, Tn, yn) - _loss(p2, bt, kind, L, H, Tg, Tn, yn)) / (2 * h)
        scale = max(1.0, abs(rec.loss))
        assert abs(fd - grad[j]) <= 2e-6 * abs(grad[j]) + 2e-7 * scale, (j, fd, grad[j])
        worst = max(worst, abs(fd - grad[j]))
    assert worst < 1e-5


def test_softplus_and_sigmoid_extremes():
    """The stable forms stay finite and exact where the naive ones overflow or
    round to zero."""
    x = np.array([-800.0, -40.0, 0.0, 40.0, 800.0])
    sp = gcl.softplus(x)
    assert np.all(np.isfinite(sp))
    assert sp[2] == pytest.approx(math.log(2.0))
    assert sp[4] == 800.0 and sp[3] == pytest.approx(40.0 + math.exp(-40.0))
    assert sp[1] == pytest.approx(math.exp(-40.0), rel=1e-12)
    sg = gcl.sigmoid(x)
    assert sg[0] == pytest.approx(0.0, abs=1e-300) and sg[4] == 1.0 and sg[2] == 0.5
    assert sg[1] == pytest.approx(math.exp(-40.0), rel=1e-12)
