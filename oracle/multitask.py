"""FP64 oracle for multitask heads (test infrastructure only).

HydraGNN, the library the paper trains with (Section 3), is multi-headed:
besides graph-level outputs computed from the pooled graph embedding it can
predict node-level quantities directly from the last GC layer's node
embeddings, and the losses of the heads are added with weights.  The paper's
model uses a single graph-level head (the HOMO-LUMO gap); this module extends
the single-head oracle in pna.py to Tg graph-level and Tn node-level heads:

  graph head t: y[b, t] = w2_t ReLU(W1_t g_b + b1_t) + b2_t, g_b the mean of
                the graph's node embeddings (as in pna.py);
  node head s:  z[i, s] = w2_s ReLU(W1_s h_i + b1_s) + b2_s for every node;
  loss = sum_t a_t mean_b (y[b,t] - Y[b,t])^2 + sum_s c_s mean_i (z[i,s] - Z[i,s])^2.

Packed parameters: the GC layers as in pna.py, then the Tg graph heads, then
the Tn node heads, each head W1 [H, H], b1 [H], w2 [1, H], b2 [1].  With one
graph head, no node head and weight 1 this is exactly pna.forward/backward.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import pna


def head_size(H: int) -> int:
    return H * H + 2 * H + 1


def unpack_heads(params, num_layers: int, hidden: int, node_feat: int, edge_feat: int,
                 Tg: int, Tn: int):
    """(layer dict in pna's names, [graph head dicts], [node head dicts])."""
    p = np.asarray(params, np.float64).copy()
    H = hidden
    nl = 0
    for l in range(num_layers):
        F = node_feat if l == 0 else H
        nl += H * (2 * F + edge_feat) + H + H * (F + 12 * H) + H
    hs = head_size(H)
    if p.shape[0] != nl + (Tg + Tn) * hs:
        raise ValueError(f"packed vector has {p.shape[0]} values, shapes need "
                         f"{nl + (Tg + Tn) * hs}")
    # reuse pna.unpack for the layers by appending a dummy head
    layers = pna.unpack(np.concatenate([p[:nl], np.zeros(hs)]), num_layers, H, node_feat,
                        edge_feat)
    for k in ("W1", "b1", "w2", "b2"):
        layers.pop(k)

    def head(off):
        return {"W1": p[off:off + H * H].reshape(H, H),
                "b1": p[off + H * H:off + H * H + H],
                "w2": p[off + H * H + H:off + H * H + 2 * H].reshape(1, H),
                "b2": p[off + H * H + 2 * H:off + hs]}

    graph = [head(nl + t * hs) for t in range(Tg)]
    node = [head(nl + (Tg + s) * hs) for s in range(Tn)]
    return layers, graph, node


@dataclasses.dataclass
class HeadsRecord:
    graph: List[dict]
    node: List[dict]
    g: np.ndarray                 # [B, H] pooled embeddings
    h: np.ndarray                 # [N, H] last GC layer's output
    gp: np.ndarray                # graph_ptr
    gpre: List[np.ndarray]        # per graph head [B, H]
    npre: List[np.ndarray]        # per node head [N, H]
    y: np.ndarray                 # [B, Tg]
    z: np.ndarray                 # [N, Tn]
    y_target: Optional[np.ndarray]
    z_target: Optional[np.ndarray]
    gw: np.ndarray
    nw: np.ndarray
    loss: Optional[float]


def heads_forward(h, graph_ptr, graph: List[dict], node: List[dict],
                  graph_weights=None, node_weights=None, y=None,
                  y_node=None) -> HeadsRecord:
    """Mean pooling, every head and the weighted loss, from the last GC
    layer's node embeddings h [N, H]."""
    h = np.asarray(h, np.float64)
    N, H = h.shape
    gp = np.asarray(graph_ptr, np.int64)
    B = gp.shape[0] - 1
    Tg, Tn = len(graph), len(node)
    g = np.zeros((B, H))
    for b in range(B):
        g[b] = h[gp[b]:gp[b + 1]].sum(0) / (gp[b + 1] - gp[b])
    gpre, ys = [], []
    for hd in graph:
        pre = g @ hd["W1"].T + hd["b1"]
        gpre.append(pre)
        ys.append((np.maximum(pre, 0.0) @ hd["w2"].T)[:, 0] + hd["b2"][0])
    npre, zs = [], []
    for hd in node:
        pre = h @ hd["W1"].T + hd["b1"]
        npre.append(pre)
        zs.append((np.maximum(pre, 0.0) @ hd["w2"].T)[:, 0] + hd["b2"][0])
    yv = np.stack(ys, 1)
    z = np.stack(zs, 1) if Tn else np.zeros((N, 0))
    gw = np.ones(Tg) if graph_weights is None else np.asarray(graph_weights, np.float64)
    nw = np.ones(Tn) if node_weights is None else np.asarray(node_weights, np.float64)
    yt = None if y is None else np.asarray(y, np.float64).reshape(-1, Tg)
    zt = None if y_node is None else np.asarray(y_node, np.float64).reshape(N, Tn)
    loss = None
    if yt is not None and (Tn == 0 or zt is not None):
        loss = float(sum(gw[t] * ((yv[:, t] - yt[:, t]) ** 2).sum() / B for t in range(Tg)))
        loss += float(sum(nw[s] * ((z[:, s] - zt[:, s]) ** 2).sum() / N for s in range(Tn)))
    return HeadsRecord(graph, node, g, h, gp, gpre, npre, yv, z, yt, zt, gw, nw, loss)


def heads_backward(hr: HeadsRecord, graph_relu=None, node_relu=None, tau: float = 0.0,
                   stats=None):
    """Adjoint of heads_forward: (dL/dh [N, H], [per-head gradient dicts])."""
    if stats is None:
        stats = {"relu": 0, "argmin": 0, "argmax": 0}
    B, Tg = hr.y.shape
    N, H = hr.h.shape
    gp = hr.gp
    dg = np.zeros((B, H))
    gheads = []
    for t, hd in enumerate(hr.graph):
        dy = 2.0 * hr.gw[t] * (hr.y[:, t] - hr.y_target[:, t]) / B
        pre = hr.gpre[t]
        mask = pna._replay_relu(pre, pre > 0, None if graph_relu is None else graph_relu[t],
                                tau, stats, f"graph head {t}")
        q = np.maximum(pre, 0.0) * mask
        dpre = dy[:, None] * hd["w2"][0][None, :] * mask
        gheads.append({"W1": dpre.T @ hr.g, "b1": dpre.sum(0), "w2": (dy @ q)[None, :],
                       "b2": np.array([dy.sum()])})
        dg += dpre @ hd["W1"]
    dh = np.zeros((N, H))
    for b in range(B):
        dh[gp[b]:gp[b + 1]] = dg[b] / (gp[b + 1] - gp[b])
    nheads = []
    for s, hd in enumerate(hr.node):
        e = 2.0 * hr.nw[s] * (hr.z[:, s] - hr.z_target[:, s]) / N
        pre = hr.npre[s]
        mask = pna._replay_relu(pre, pre > 0, None if node_relu is None else node_relu[s],
                                tau, stats, f"node head {s}")
        q = np.maximum(pre, 0.0) * mask
        dpre = e[:, None] * hd["w2"][0][None, :] * mask
        nheads.append({"W1": dpre.T @ hr.h, "b1": dpre.sum(0), "w2": (e @ q)[None, :],
                       "b2": np.array([e.sum()])})
        dh += dpre @ hd["W1"]
    return dh, gheads + nheads


@dataclasses.dataclass
class MTRecord:
    base: pna.ForwardRecord       # GC stack, pooling; its head fields unused
    heads: HeadsRecord

    # the head fields under their earlier names
    @property
    def y(self):
        return self.heads.y

    @property
    def z(self):
        return self.heads.z

    @property
    def loss(self):
        return self.heads.loss

    @property
    def g(self):
        return self.heads.g


def forward(params, batch, num_layers: int, hidden: int, delta: float, Tg: int, Tn: int,
            graph_weights: Optional[Sequence[float]] = None,
            node_weights: Optional[Sequence[float]] = None,
            y_node: Optional[np.ndarray] = None, eps: float = pna.STD_EPS) -> MTRecord:
    """Forward of the GC stack and all heads; batch.y is [B, Tg] (or [B] for Tg = 1)."""
    x = np.asarray(batch.x, np.float64)
    N, F0 = x.shape
    Fe = 0 if batch.edge_attr is None else batch.edge_attr.shape[1]
    layers, graph, node = unpack_heads(params, num_layers, hidden, F0, Fe, Tg, Tn)
    # the GC stack through pna.forward with a zero single head (its outputs unused)
    single = pna.pack({**layers, "W1": np.zeros((hidden, hidden)), "b1": np.zeros(hidden),
                       "w2": np.zeros((1, hidden)), "b2": np.zeros(1)}, num_layers)
    base = pna.forward(single, batch, num_layers, hidden, delta, eps, with_loss=False)
    hr = heads_forward(base.layers[-1].h_out, batch.graph_ptr, graph, node, graph_weights,
                       node_weights, batch.y, y_node)
    return MTRecord(base, hr)


def backward(rec: MTRecord, hint: Optional[pna.Decisions] = None,
             graph_relu: Optional[List[np.ndarray]] = None,
             node_relu: Optional[List[np.ndarray]] = None, tau: float = 0.0):
    """Gradient of the weighted loss w.r.t. the packed parameters and x.

    ``hint`` replays the GC stack's decisions (pna.Decisions, head_relu
    ignored); ``graph_relu``/``node_relu`` replay the heads' ReLU decisions.
    Returns (packed gradient, dx, adopted-decision counts).
    """
    base = rec.base
    L = base.cfg["num_layers"]
    stats = {"relu": 0, "argmin": 0, "argmax": 0}
    dh, hgrads = heads_backward(rec.heads, graph_relu, node_relu, tau, stats)
    G: Dict[str, np.ndarray] = {}
    dx = pna.layers_backward(base, dh, G, hint, tau, stats)
    keys = []
    for l in range(L):
        keys += [f"l{l}.Wm", f"l{l}.bm", f"l{l}.Wp", f"l{l}.bp"]
    parts = [G[k].ravel() for k in keys]
    for hd in hgrads:
        parts += [hd[k].ravel() for k in ("W1", "b1", "w2", "b2")]
    return np.concatenate(parts), dx, stats
