"""Pins of the multitask-head oracle (oracle/multitask.py), host only.

* one graph head, no node head, weight 1: exactly the single-head oracle;
* central finite differences of the weighted loss w.r.t. every parameter;
* the heads and the weighted loss re-expressed in float64 torch autograd on
  top of the GC stack's node embeddings;
* node heads are equivariant under node permutations within graphs.
"""
import numpy as np
import pytest

import oracle
from oracle import multitask as mt
from paper_2207_11333_amd import synth


def _case(seed, Tg, Tn, B=4, H=4, L=2, fe=1):
    b = synth.make_batch(seed, B, 3, 8, fe)
    rng = np.random.default_rng(seed + 7)
    shape = synth.ModelShape(L, H, 9, fe)
    layers = synth.init_params(shape, seed).astype(np.float64)
    nl = layers.shape[0] - mt.head_size(H)
    heads = rng.uniform(-0.5, 0.5, size=(Tg + Tn) * mt.head_size(H))
    params = np.concatenate([layers[:nl], heads])
    y = rng.normal(5.0, 1.5, size=(B, Tg))
    yn = rng.normal(0.0, 1.0, size=(b.num_nodes, Tn))
    b = synth.Batch(b.graph_ptr, b.x, b.edge_index, b.edge_attr, y.astype(np.float32))
    return b, params, yn, L, H


def test_single_graph_head_is_the_plain_oracle():
    b0 = synth.make_batch(5, 6, 4, 12, 1)
    L, H = 2, 6
    params = synth.init_params(synth.ModelShape(L, H, 9, 1), 5).astype(np.float64)
    ref = oracle.forward(params, b0, L, H, 1.2)
    g_ref, dx_ref, _ = oracle.backward(ref)
    rec = mt.forward(params, b0, L, H, 1.2, 1, 0)
    g, dx, _ = mt.backward(rec)
    np.testing.assert_array_equal(rec.y[:, 0], ref.y)
    assert rec.loss == ref.loss
    np.testing.assert_array_equal(g, g_ref)
    np.testing.assert_array_equal(dx, dx_ref)


def _decisions(rec):
    out = [p > 0 for p in rec.heads.gpre] + [p > 0 for p in rec.heads.npre]
    for lr in rec.base.layers:
        out += [lr.u > 0, lr.argmin, lr.argmax]
    return out


@pytest.mark.parametrize("seed,Tg,Tn", [(71, 2, 2), (72, 1, 3), (73, 3, 0)])
def test_multitask_gradients_central_fd(seed, Tg, Tn):
    b, params, yn, L, H = _case(seed, Tg, Tn)
    gw = [0.5, 2.0, 1.0][:Tg]
    nw = [1.5, 0.25, 1.0][:Tn]
    fwd = lambda p: mt.forward(p, b, L, H, 1.0, Tg, Tn, gw, nw, yn)
    rec = fwd(params)
    grad, _, _ = mt.backward(rec)
    base = _decisions(rec)
    checked = 0
    for j in range(params.shape[0]):
        hstep = 1e-6 * max(1.0, abs(params[j]))
        pp = params.copy(); pp[j] += hstep
        pm = params.copy(); pm[j] -= hstep
        rp, rm = fwd(pp), fwd(pm)
        if not all(np.array_equal(a, c) for a, c in zip(base, _decisions(rp))) or \
           not all(np.array_equal(a, c) for a, c in zip(base, _decisions(rm))):
            continue
        fd = (rp.loss - rm.loss) / (2 * hstep)
        assert fd == pytest.approx(grad[j], rel=2e-6, abs=2e-7 * max(1, abs(rec.loss))), j
        checked += 1
    assert checked > 0.9 * params.shape[0]


@pytest.mark.parametrize("seed,Tg,Tn", [(81, 2, 2), (82, 1, 1)])
def test_heads_against_torch_autograd(seed, Tg, Tn):
    import torch
    b, params, yn, L, H = _case(seed, Tg, Tn, B=6, H=5)
    gw, nw = [0.7, 1.3][:Tg], [2.0, 0.5][:Tn]
    rec = mt.forward(params, b, L, H, 1.0, Tg, Tn, gw, nw, yn)
    grad, _, _ = mt.backward(rec)
    hs = mt.head_size(H)
    heads = torch.tensor(params[-(Tg + Tn) * hs:], requires_grad=True)
    h = torch.tensor(rec.base.layers[-1].h_out, requires_grad=True)
    gp = torch.tensor(b.graph_ptr, dtype=torch.int64)
    B = gp.shape[0] - 1
    seg = torch.repeat_interleave(torch.arange(B), gp[1:] - gp[:-1])
    g = torch.zeros(B, H, dtype=torch.float64).index_add_(0, seg, h)
    g = g / (gp[1:] - gp[:-1]).to(torch.float64)[:, None]
    lin = torch.nn.functional.linear
    loss = 0
    for k in range(Tg + Tn):
        p = heads[k * hs:(k + 1) * hs]
        W1, b1 = p[:H * H].view(H, H), p[H * H:H * H + H]
        w2, b2 = p[H * H + H:H * H + 2 * H].view(1, H), p[H * H + 2 * H:]
        inp = g if k < Tg else h
        out = lin(torch.relu(lin(inp, W1, b1)), w2, b2)[:, 0]
        if k < Tg:
            t = torch.tensor(np.asarray(b.y, np.float64)[:, k])
            loss = loss + gw[k] * torch.mean((out - t) ** 2)
        else:
            t = torch.tensor(yn[:, k - Tg])
            loss = loss + nw[k - Tg] * torch.mean((out - t) ** 2)
    loss.backward()
    assert loss.item() == pytest.approx(rec.loss, rel=1e-12)
    np.testing.assert_allclose(heads.grad.numpy(), grad[-(Tg + Tn) * hs:], rtol=1e-10,
                               atol=1e-12)


def test_node_heads_permutation_equivariant():
    b, params, yn, L, H = _case(91, 1, 2, B=5)
    rec = mt.forward(params, b, L, H, 1.0, 1, 2, None, None, yn)
    rng = np.random.default_rng(3)
    pi = np.arange(b.num_nodes)
    for g in range(b.num_graphs):
        lo, hi = b.graph_ptr[g], b.graph_ptr[g + 1]
        pi[lo:hi] = lo + rng.permutation(hi - lo)
    inv = np.argsort(pi)
    b2 = synth.Batch(b.graph_ptr, b.x[inv], pi[b.edge_index].astype(np.int32), b.edge_attr, b.y)
    rec2 = mt.forward(params, b2, L, H, 1.0, 1, 2, None, None, yn[inv])
    np.testing.assert_allclose(rec2.z[pi], rec.z, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(rec2.y, rec.y, rtol=1e-12)
    assert rec2.loss == pytest.approx(rec.loss, rel=1e-12)
