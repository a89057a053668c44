"""FP64 oracle for the other GC layer kinds: GraphSAGE and CGCNN (test
infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline may use it; the product path never does).

The paper's background on graph convolutional networks (Section 2) names
three GC layer kinds implemented in HydraGNN -- PNA, crystal-graph CGCNN and
GraphSAGE -- and runs its experiments with PNA (pna.py).  The other two are
taken from their original formulations:

GraphSAGE, mean aggregator (Hamilton, Ying and Leskovec, 2017):
    M_i  = mean of h_j over the in-edges j -> i (one term per edge; 0 for a
           node without in-edges),
    h'_i = ReLU(W_self h_i + W_nbr M_i + b),
  without the optional L2 normalisation of the output.  Packed per layer:
  W [H, 2F] = [W_self | W_nbr] (row-major), then b [H].

CGCNN (Xie and Grossman, 2018):
    h^0  = W_emb x + b_emb            (a linear atom embedding, no activation)
    z_ij = [h_i || h_j || e_ij]       for every in-edge j -> i
    f    = W_f z_ij + b_f,  s = W_s z_ij + b_s
    h'_i = ReLU(h_i + sum over in-edges of sigmoid(f) * softplus(s)).
  The filter (f) and core (s) linears are packed as one [2H, 2H + Fe] matrix,
  rows 0..H-1 for f and H..2H-1 for s, and one [2H] bias.  Packed: W_emb
  [H, F0], b_emb [H], then per layer W [2H, 2H + Fe], b [2H].

Readings where the sources leave a choice: every GC layer ends in ReLU, as in
the PNA stack here (the original CGCNN applies softplus after the residual
sum, and both originals offer batch normalisation, whose batch statistics
are left out as for PNA so that a graph's output does not depend on the
other graphs of its batch); in-edges are taken in the canonical (source id,
edge id) order; ReLU'(0) = 0.  After the GC stack come the same mean pooling,
graph-level and node-level heads and weighted loss as multitask.py (packed
after the layers: graph heads, then node heads).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

from . import multitask, pna

SAGE = "sage"
CGCNN = "cgcnn"
KINDS = (SAGE, CGCNN)


# --------------------------------------------------------------------------
# packing
# --------------------------------------------------------------------------

def layer_shapes(kind: str, num_layers: int, hidden: int, node_feat: int, edge_feat: int):
    """[(name, shape)] of the GC stack in packing order."""
    H, Fe = hidden, edge_feat
    out = []
    if kind == SAGE:
        for l in range(num_layers):
            F = node_feat if l == 0 else H
            out += [(f"l{l}.W", (H, 2 * F)), (f"l{l}.b", (H,))]
    elif kind == CGCNN:
        out += [("emb.W", (H, node_feat)), ("emb.b", (H,))]
        for l in range(num_layers):
            out += [(f"l{l}.W", (2 * H, 2 * H + Fe)), (f"l{l}.b", (2 * H,))]
    else:
        raise ValueError(f"unknown layer kind {kind!r}")
    return out


def stack_size(kind, num_layers, hidden, node_feat, edge_feat) -> int:
    return int(sum(int(np.prod(s)) for _, s in
                   layer_shapes(kind, num_layers, hidden, node_feat, edge_feat)))


def unpack(params, kind, num_layers, hidden, node_feat, edge_feat, Tg, Tn):
    """(GC stack dict, [graph head dicts], [node head dicts]) as float64."""
    p = np.asarray(params, np.float64).copy()
    shapes = layer_shapes(kind, num_layers, hidden, node_feat, edge_feat)
    nl = stack_size(kind, num_layers, hidden, node_feat, edge_feat)
    hs = multitask.head_size(hidden)
    if p.shape[0] != nl + (Tg + Tn) * hs:
        raise ValueError(f"packed vector has {p.shape[0]} values, shapes need "
                         f"{nl + (Tg + Tn) * hs}")
    P, off = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        P[name] = p[off:off + n].reshape(shp)
        off += n
    H = hidden

    def head(o):
        return {"W1": p[o:o + H * H].reshape(H, H), "b1": p[o + H * H:o + H * H + H],
                "w2": p[o + H * H + H:o + H * H + 2 * H].reshape(1, H),
                "b2": p[o + H * H + 2 * H:o + hs]}

    graph = [head(nl + t * hs) for t in range(Tg)]
    node = [head(nl + (Tg + s) * hs) for s in range(Tn)]
    return P, graph, node


# --------------------------------------------------------------------------
# elementwise functions (FP64)
# --------------------------------------------------------------------------

def sigmoid(x):
    x = np.asarray(x, np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def softplus(x):
    """ln(1 + e^x), written so that it neither overflows nor loses small values."""
    x = np.asarray(x, np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------

@dataclasses.dataclass
class GCLayerRecord:
    h_in: np.ndarray                    # [N, F]
    u: np.ndarray                       # [N, H] pre-activation
    h_out: np.ndarray                   # [N, H]
    M: Optional[np.ndarray] = None      # SAGE: neighbour means [N, F]
    z: Optional[np.ndarray] = None      # CGCNN: per CSR edge [h_i || h_j || e] [E, 2H+Fe]
    f: Optional[np.ndarray] = None      # CGCNN: filter pre-activation [E, H]
    s: Optional[np.ndarray] = None      # CGCNN: core pre-activation [E, H]


@dataclasses.dataclass
class GCRecord:
    kind: str
    cfg: dict
    P: Dict[str, np.ndarray]
    csr: pna.CSR
    x: np.ndarray
    h0: Optional[np.ndarray]            # CGCNN embedding output
    layers: List[GCLayerRecord]
    heads: multitask.HeadsRecord

    @property
    def y(self):
        return self.heads.y

    @property
    def z(self):
        return self.heads.z

    @property
    def loss(self):
        return self.heads.loss


def _csr_dst(csr: pna.CSR) -> np.ndarray:
    """Destination of every CSR position."""
    N = csr.deg.shape[0]
    return np.repeat(np.arange(N), np.asarray(csr.deg, np.int64))


def sage_layer(W, b, h, csr: pna.CSR) -> GCLayerRecord:
    N, F = h.shape
    M = np.zeros((N, F))
    for i in range(N):
        lo, hi = int(csr.rowptr[i]), int(csr.rowptr[i + 1])
        if hi > lo:
            M[i] = h[csr.csr_src[lo:hi]].sum(0) / (hi - lo)
    u = h @ W[:, :F].T + M @ W[:, F:].T + b
    return GCLayerRecord(h_in=h, u=u, h_out=np.maximum(u, 0.0), M=M)


def cgcnn_layer(W, b, h, csr: pna.CSR, e_csr) -> GCLayerRecord:
    N, H = h.shape
    dst = _csr_dst(csr)
    src = np.asarray(csr.csr_src, np.int64)
    parts = [h[dst], h[src]]
    if e_csr is not None:
        parts.append(e_csr)
    z = np.concatenate(parts, 1)
    pre = z @ W.T + b
    f, s = pre[:, :H], pre[:, H:]
    msg = sigmoid(f) * softplus(s)
    agg = np.zeros((N, H))
    for i in range(N):
        lo, hi = int(csr.rowptr[i]), int(csr.rowptr[i + 1])
        if hi > lo:
            agg[i] = msg[lo:hi].sum(0)
    u = h + agg
    return GCLayerRecord(h_in=h, u=u, h_out=np.maximum(u, 0.0), z=z, f=f, s=s)


def forward(params, batch, kind: str, num_layers: int, hidden: int, Tg: int = 1,
            Tn: int = 0, graph_weights=None, node_weights=None, y_node=None,
            max_degree: int = 255) -> GCRecord:
    """GC stack of the given kind, pooling, heads and loss; batch.y [B] or [B, Tg]."""
    x = np.asarray(batch.x, np.float64)
    N, F0 = x.shape
    ea = batch.edge_attr
    Fe = 0 if ea is None else ea.shape[1]
    pna.check_batch(batch.graph_ptr, batch.edge_index, N, max_degree)
    P, graph, node = unpack(params, kind, num_layers, hidden, F0, Fe, Tg, Tn)
    csr = pna.csr_build(batch.graph_ptr, batch.edge_index, N)
    e_csr = None if ea is None else np.asarray(ea, np.float64)[np.asarray(csr.csr_eid)]
    h0 = None
    h = x
    if kind == CGCNN:
        h0 = x @ P["emb.W"].T + P["emb.b"]
        h = h0
    layers = []
    for l in range(num_layers):
        if kind == SAGE:
            rec = sage_layer(P[f"l{l}.W"], P[f"l{l}.b"], h, csr)
        else:
            rec = cgcnn_layer(P[f"l{l}.W"], P[f"l{l}.b"], h, csr, e_csr)
        layers.append(rec)
        h = rec.h_out
    hr = multitask.heads_forward(h, batch.graph_ptr, graph, node, graph_weights,
                                 node_weights, batch.y, y_node)
    cfg = dict(num_layers=num_layers, hidden=hidden, node_feat=F0, edge_feat=Fe, Tg=Tg,
               Tn=Tn)
    return GCRecord(kind, cfg, P, csr, x, h0, layers, hr)


# --------------------------------------------------------------------------
# backward (hand-written adjoints)
# --------------------------------------------------------------------------

def sage_layer_backward(W, rec: GCLayerRecord, du, csr: pna.CSR):
    """(dW, db, dh_in) from du = dL/du (the ReLU adjoint already applied)."""
    F = rec.h_in.shape[1]
    dW = np.concatenate([du.T @ rec.h_in, du.T @ rec.M], 1)
    db = du.sum(0)
    dh = du @ W[:, :F]
    dM = du @ W[:, F:]
    for i in range(dM.shape[0]):
        lo, hi = int(csr.rowptr[i]), int(csr.rowptr[i + 1])
        for q in range(lo, hi):
            dh[csr.csr_src[q]] += dM[i] / (hi - lo)
    return dW, db, dh


def cgcnn_layer_backward(W, rec: GCLayerRecord, du, csr: pna.CSR):
    """(dW, db, dh_in) from du = dL/du; the residual passes du to h_in."""
    H = du.shape[1]
    dst = _csr_dst(csr)
    src = np.asarray(csr.csr_src, np.int64)
    sf = sigmoid(rec.f)
    dmsg = du[dst]                               # d(sum)/d(msg) = 1 per edge
    df = dmsg * softplus(rec.s) * sf * (1.0 - sf)
    ds = dmsg * sf * sigmoid(rec.s)              # softplus' = sigmoid
    dpre = np.concatenate([df, ds], 1)           # [E, 2H]
    dW = dpre.T @ rec.z
    db = dpre.sum(0)
    dz = dpre @ W                                # [E, 2H + Fe]
    dh = du.copy()
    np.add.at(dh, dst, dz[:, :H])
    np.add.at(dh, src, dz[:, H:2 * H])
    return dW, db, dh


def backward(rec: GCRecord, relu_hint: Optional[List[Optional[np.ndarray]]] = None,
             graph_relu=None, node_relu=None, tau: float = 0.0):
    """Gradient of the loss w.r.t. the packed parameters.

    ``relu_hint[l]`` (the [N, H] boolean h_out > 0 of another implementation)
    and ``graph_relu``/``node_relu`` are adopted where they differ from this
    oracle's own decisions only inside the tie window ``tau`` (see pna.py).
    Returns (packed gradient, adopted-decision counts).
    """
    stats = {"relu": 0, "argmin": 0, "argmax": 0}
    dh, hgrads = multitask.heads_backward(rec.heads, graph_relu, node_relu, tau, stats)
    L = rec.cfg["num_layers"]
    G: Dict[str, np.ndarray] = {}
    for l in range(L - 1, -1, -1):
        lr = rec.layers[l]
        mask = pna._replay_relu(lr.u, lr.u > 0, None if relu_hint is None else relu_hint[l],
                                tau, stats, f"layer {l}")
        du = dh * mask
        W = rec.P[f"l{l}.W"]
        if rec.kind == SAGE:
            dW, db, dh = sage_layer_backward(W, lr, du, rec.csr)
        else:
            dW, db, dh = cgcnn_layer_backward(W, lr, du, rec.csr)
        G[f"l{l}.W"], G[f"l{l}.b"] = dW, db
    if rec.kind == CGCNN:
        G["emb.W"] = dh.T @ rec.x
        G["emb.b"] = dh.sum(0)
    cfg = rec.cfg
    shapes = layer_shapes(rec.kind, L, cfg["hidden"], cfg["node_feat"], cfg["edge_feat"])
    parts = [G[name].ravel() for name, _ in shapes]
    for hd in hgrads:
        parts += [hd[k].ravel() for k in ("W1", "b1", "w2", "b2")]
    return np.concatenate(parts), stats

