"""FP64 CPU oracle for the PNA-style GCNN hot path (test infrastructure only).

This is the plain, slow, obviously-correct reference against which the HIP
path is checked.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.

What it computes (Choi et al., "Scalable training of graph convolutional
neural networks for fast and accurate predictions of HOMO-LUMO gap in
molecules"):
  * GC layers that pass messages between bonded atoms and use node degree
    (Section 3.1), of the PNA kind (Section 3.1 and Section 5.1, 6 layers);
    the paper only names PNA, so the layer is read as: message
    m_k = W^m [h_dst || h_src || e_k] + b^m; per destination the aggregators
    mean, min, max and std (sqrt(population variance + eps)); degree scalers
    identity, s+ = ln(d+1)/delta and s- = delta/ln(d+1); update
    h' = ReLU(W^p [h || A || s+ A || s- A] + b^p), A = [mean||min||max||std].
  * global mean pooling over each graph's nodes (Section 3.1),
  * fully connected head Linear(H,H)-ReLU-Linear(H,1) (Section 3.1, 3.2),
  * MSE loss averaged over the graphs of the batch (Section 3.2),
  * the backward pass of every step (Section 3.2) written out by hand,
  * AdamW (Section 5.1, lr 1e-3), decoupled weight decay, t starting at 1.
Conventions where the paper is silent: canonical in-edge order per node is
(source id, edge id); a min/max subgradient goes wholly to the first edge in
that order attaining the extremum; ReLU'(0) = 0; a node with no in-edge has
A = 0 and s+ = s- = 0; an empty graph is an error.

Every array is float64 internally.  Parameters use the packed interchange
order: per layer W^m [H, 2F+Fe], b^m [H], W^p [H, F+12H], b^p [H]; then
W1 [H, H], b1 [H], w2 [1, H], b2 [1] (row-major [out, in]).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

STD_EPS = 1e-5


class DecisionMismatch(AssertionError):
    """A decision supplied for replay is not within the tie window."""


# --------------------------------------------------------------------------
# parameter packing
# --------------------------------------------------------------------------

def unpack(params: np.ndarray, num_layers: int, hidden: int, node_feat: int,
           edge_feat: int) -> Dict[str, np.ndarray]:
    """Split the packed vector into named float64 arrays (views of a copy)."""
    p = np.asarray(params, dtype=np.float64).copy()
    H, Fe = hidden, edge_feat
    out, off = {}, 0

    def take(name, shape):
        nonlocal off
        n = int(np.prod(shape))
        out[name] = p[off:off + n].reshape(shape)
        off += n

    for l in range(num_layers):
        F = node_feat if l == 0 else H
        take(f"l{l}.Wm", (H, 2 * F + Fe))
        take(f"l{l}.bm", (H,))
        take(f"l{l}.Wp", (H, F + 12 * H))
        take(f"l{l}.bp", (H,))
    take("W1", (H, H))
    take("b1", (H,))
    take("w2", (1, H))
    take("b2", (1,))
    if off != p.shape[0]:
        raise ValueError(f"packed vector has {p.shape[0]} values, shapes need {off}")
    return out


def pack(named: Dict[str, np.ndarray], num_layers: int) -> np.ndarray:
    keys = []
    for l in range(num_layers):
        keys += [f"l{l}.Wm", f"l{l}.bm", f"l{l}.Wp", f"l{l}.bp"]
    keys += ["W1", "b1", "w2", "b2"]
    return np.concatenate([np.asarray(named[k], np.float64).ravel() for k in keys])


# --------------------------------------------------------------------------
# batch checks and the destination-sorted CSR (Table 1 layout in)
# --------------------------------------------------------------------------

def check_batch(graph_ptr, edge_index, num_nodes: int, max_degree: int) -> None:
    """Raise ValueError for every malformed-batch condition of the contract."""
    gp = np.asarray(graph_ptr, dtype=np.int64)
    ei = np.asarray(edge_index, dtype=np.int64)
    if gp.ndim != 1 or gp.shape[0] < 1 or gp[0] != 0 or gp[-1] != num_nodes:
        raise ValueError("graph_ptr must run from 0 to num_nodes")
    if np.any(np.diff(gp) <= 0):
        raise ValueError("empty graph in batch")
    if ei.ndim != 2 or ei.shape[0] != 2:
        raise ValueError("edge_index must have shape (2, E)")
    src, dst = ei
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= num_nodes
                     or dst.max() >= num_nodes):
        raise ValueError("edge endpoint out of range")
    node_graph = np.repeat(np.arange(gp.shape[0] - 1), np.diff(gp))
    if src.size and np.any(node_graph[src] != node_graph[dst]):
        raise ValueError("edge crosses graphs")
    if src.size and (np.bincount(dst, minlength=num_nodes).max() > max_degree
                     or np.bincount(src, minlength=num_nodes).max() > max_degree):
        raise ValueError("degree above max_degree")


@dataclasses.dataclass
class CSR:
    rowptr: np.ndarray    # [N+1] in-edge segment offsets
    csr_src: np.ndarray   # [E] source of the q-th edge in (dst, src, eid) order
    csr_eid: np.ndarray   # [E] original edge id of the q-th edge
    deg: np.ndarray       # [N] in-degree
    srcptr: np.ndarray    # [N+1] out-edge segment offsets
    t2csr: np.ndarray     # [E] CSR positions of each source's out-edges, ascending
    node_graph: np.ndarray  # [N] graph id of each node


def csr_build(graph_ptr, edge_index, num_nodes: int) -> CSR:
    """Sort edges by (dst, src, eid) and build the by-source transpose."""
    ei = np.asarray(edge_index, dtype=np.int64)
    src, dst = ei
    E = src.shape[0]
    eid = np.arange(E)
    order = np.lexsort((eid, src, dst))
    deg = np.bincount(dst, minlength=num_nodes)
    rowptr = np.concatenate([[0], np.cumsum(deg)])
    csr_src = src[order]
    # transpose: CSR positions q grouped by their source, ascending q
    tord = np.lexsort((np.arange(E), csr_src))
    odeg = np.bincount(src, minlength=num_nodes)
    srcptr = np.concatenate([[0], np.cumsum(odeg)])
    gp = np.asarray(graph_ptr, dtype=np.int64)
    node_graph = np.repeat(np.arange(gp.shape[0] - 1), np.diff(gp))
    i32 = lambda a: np.asarray(a, dtype=np.int32)
    return CSR(i32(rowptr), i32(csr_src), i32(order), i32(deg), i32(srcptr),
               i32(tord), i32(node_graph))


def degree_scalers(deg: np.ndarray, delta: float):
    """s+ = ln(d+1)/delta and s- = delta/ln(d+1); both 0 where d = 0."""
    d = np.asarray(deg, dtype=np.float64)
    lg = np.log(d + 1.0)
    sp = np.where(d > 0, lg / delta, 0.0)
    sm = np.where(d > 0, delta / np.where(d > 0, lg, 1.0), 0.0)
    return sp, sm


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------

@dataclasses.dataclass
class LayerRecord:
    h_in: np.ndarray      # [N, F]
    z: np.ndarray         # [E, 2F+Fe] message input per edge
    m: np.ndarray         # [E, H] messages
    A: np.ndarray         # [N, 4H] = [mean || min || max || std]
    argmin: np.ndarray    # [N, H] offset inside the node's in-edge segment
    argmax: np.ndarray    # [N, H]
    a: np.ndarray         # [N, F+12H] update input
    u: np.ndarray         # [N, H] pre-activation
    h_out: np.ndarray     # [N, H]


@dataclasses.dataclass
class ForwardRecord:
    cfg: dict
    P: Dict[str, np.ndarray]
    csr: CSR
    sp: np.ndarray
    sm: np.ndarray
    layers: List[LayerRecord]
    g: np.ndarray         # [B, H] pooled
    pre: np.ndarray       # [B, H] head pre-activation
    q: np.ndarray         # [B, H]
    y: np.ndarray         # [B] predictions
    target: Optional[np.ndarray]
    loss: Optional[float]
    graph_ptr: np.ndarray
    edge_index: np.ndarray


def _segment_stats(m, csr: CSR, N: int, H: int, eps: float):
    """Per destination, over its in-edges in canonical order."""
    A = np.zeros((N, 4 * H))
    amin = np.zeros((N, H), dtype=np.int64)
    amax = np.zeros((N, H), dtype=np.int64)
    for i in range(N):
        lo, hi = int(csr.rowptr[i]), int(csr.rowptr[i + 1])
        if hi == lo:
            continue
        ms = m[csr.csr_eid[lo:hi]]            # [d, H]
        d = hi - lo
        mu = ms.sum(0) / d
        var = ((ms - mu) ** 2).sum(0) / d
        A[i, 0:H] = mu
        A[i, H:2 * H] = ms.min(0)
        A[i, 2 * H:3 * H] = ms.max(0)
        A[i, 3 * H:4 * H] = np.sqrt(var + eps)
        amin[i] = ms.argmin(0)                # numpy returns the first extremum
        amax[i] = ms.argmax(0)
    return A, amin, amax


def layer_forward(Wm, bm, Wp, bp, h, edge_index, edge_attr, csr: CSR, sp, sm,
                  eps: float = STD_EPS) -> LayerRecord:
    h = np.asarray(h, np.float64)
    N = h.shape[0]
    H = bm.shape[0]
    src = np.asarray(edge_index[0], np.int64)
    dst = np.asarray(edge_index[1], np.int64)
    parts = [h[dst], h[src]]
    if edge_attr is not None:
        parts.append(np.asarray(edge_attr, np.float64))
    z = np.concatenate(parts, 1)
    m = z @ Wm.T + bm
    A, amin, amax = _segment_stats(m, csr, N, H, eps)
    a = np.concatenate([h, A, sp[:, None] * A, sm[:, None] * A], 1)
    u = a @ Wp.T + bp
    return LayerRecord(h, z, m, A, amin, amax, a, u, np.maximum(u, 0.0))


def forward(params, batch, num_layers: int, hidden: int, delta: float,
            eps: float = STD_EPS, max_degree: int = 255,
            with_loss: bool = True) -> ForwardRecord:
    """Full forward: L GC layers, mean pooling, MLP head and MSE loss.

    ``batch`` needs graph_ptr, x, edge_index, edge_attr (or None) and y.
    """
    x = np.asarray(batch.x, np.float64)
    N, F0 = x.shape
    ea = batch.edge_attr
    Fe = 0 if ea is None else ea.shape[1]
    check_batch(batch.graph_ptr, batch.edge_index, N, max_degree)
    P = unpack(params, num_layers, hidden, F0, Fe)
    csr = csr_build(batch.graph_ptr, batch.edge_index, N)
    sp, sm = degree_scalers(csr.deg, delta)
    h = x
    layers = []
    for l in range(num_layers):
        rec = layer_forward(P[f"l{l}.Wm"], P[f"l{l}.bm"], P[f"l{l}.Wp"],
                            P[f"l{l}.bp"], h, batch.edge_index, ea, csr, sp, sm, eps)
        layers.append(rec)
        h = rec.h_out
    gp = np.asarray(batch.graph_ptr, np.int64)
    B = gp.shape[0] - 1
    g = np.zeros((B, hidden))
    for b in range(B):
        g[b] = h[gp[b]:gp[b + 1]].sum(0) / (gp[b + 1] - gp[b])
    pre = g @ P["W1"].T + P["b1"]
    q = np.maximum(pre, 0.0)
    y = (q @ P["w2"].T)[:, 0] + P["b2"][0]
    target = None if batch.y is None else np.asarray(batch.y, np.float64)
    loss = None
    if with_loss and target is not None:
        loss = float(((y - target) ** 2).sum() / B)
    cfg = dict(num_layers=num_layers, hidden=hidden, node_feat=F0, edge_feat=Fe,
               delta=delta, eps=eps)
    return ForwardRecord(cfg, P, csr, sp, sm, layers, g, pre, q, y, target, loss,
                         gp, np.asarray(batch.edge_index, np.int64))


# --------------------------------------------------------------------------
# backward (hand-written adjoint) with optional decision replay
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Decisions:
    """Decisions taken by another implementation, offered for replay.

    Each entry may be None.  ``argmin[l]``/``argmax[l]`` are [N, H] segment
    offsets, ``relu[l]`` is the [N, H] boolean (h_out > 0) of layer l and
    ``head_relu`` the [B, H] boolean of the head's hidden layer.
    """
    argmin: List[Optional[np.ndarray]]
    argmax: List[Optional[np.ndarray]]
    relu: List[Optional[np.ndarray]]
    head_relu: Optional[np.ndarray] = None


def _rms(a):
    return float(np.sqrt(np.mean(np.square(a)))) if a.size else 0.0


def _replay_relu(u, own, hint, tau, stats, what):
    """Adopt ``hint`` where it differs from ``own`` only inside the tie window."""
    if hint is None:
        return own
    hint = np.asarray(hint, bool)
    diff = hint != own
    if not diff.any():
        return own
    # a ReLU decision is a tie of u against 0, so the window is measured on
    # the scale of u's own tensor: |u| <= tau * rms(u)
    bad = diff & (np.abs(u) > tau * _rms(u))
    if bad.any():
        idx = np.argwhere(bad)[0]
        raise DecisionMismatch(f"{what}: ReLU decision differs at {tuple(idx)} with "
                               f"u={u[tuple(idx)]!r} outside the tie window")
    stats["relu"] += int(diff.sum())
    return hint


def _replay_arg(vals_seg_fn, own, hint, tau, m_rms, stats, what, kind):
    """Replay argmin/argmax offsets; ``vals_seg_fn(i)`` gives the [d, H] values."""
    if hint is None:
        return own
    hint = np.asarray(hint, np.int64)
    diff = np.argwhere(hint != own)
    out = own.copy()
    for i, c in diff:
        ms = vals_seg_fn(i)
        d = ms.shape[0]
        j = int(hint[i, c])
        if not 0 <= j < d:
            raise DecisionMismatch(f"{what}: {kind} offset {j} outside segment of {d}")
        best = ms[own[i, c], c]
        gap = abs(ms[j, c] - best)
        if gap > tau * max(abs(best), m_rms):
            raise DecisionMismatch(f"{what}: {kind} at node {i} feature {c}: offset {j}"
                                   f" is {gap!r} from the extremum, outside the window")
        out[i, c] = j
        stats[kind] += 1
    return out


def backward(rec: ForwardRecord, dpred: Optional[np.ndarray] = None,
             hint: Optional[Decisions] = None, tau: float = 0.0):
    """Gradients of the loss (or of sum(dpred * y)) w.r.t. params and x.

    Returns (packed gradient [P], dx [N, F0], adopted-decision counts).
    """
    cfg, P, csr = rec.cfg, rec.P, rec.csr
    L, H = cfg["num_layers"], cfg["hidden"]
    B = rec.y.shape[0]
    gp = rec.graph_ptr
    stats = {"relu": 0, "argmin": 0, "argmax": 0}
    G = {}
    if dpred is None:
        dy = 2.0 * (rec.y - rec.target) / B
    else:
        dy = np.asarray(dpred, np.float64)
    # head: y = w2 q + b2, q = relu(pre), pre = W1 g + b1
    G["w2"] = (dy @ rec.q)[None, :]
    G["b2"] = np.array([dy.sum()])
    mask = _replay_relu(rec.pre, rec.pre > 0,
                        None if hint is None else hint.head_relu, tau, stats, "head")
    dpre = dy[:, None] * P["w2"][0][None, :] * mask
    G["W1"] = dpre.T @ rec.g
    G["b1"] = dpre.sum(0)
    dg = dpre @ P["W1"]
    N = rec.layers[0].h_in.shape[0]
    dh = np.zeros((N, H))
    for b in range(B):
        dh[gp[b]:gp[b + 1]] = dg[b] / (gp[b + 1] - gp[b])
    dh = layers_backward(rec, dh, G, hint, tau, stats)
    return pack(G, L), dh, stats


def layers_backward(rec, dh, G, hint: Optional[Decisions], tau: float, stats):
    """Adjoint of the GC stack: from dL/dh of the last layer's output, fill the
    layer gradients into G and return dL/dx (Section 3.2, backward phase)."""
    cfg, P, csr = rec.cfg, rec.P, rec.csr
    L, H = cfg["num_layers"], cfg["hidden"]
    N = rec.layers[0].h_in.shape[0]
    src, dst = rec.edge_index
    for l in reversed(range(L)):
        lr = rec.layers[l]
        F = lr.h_in.shape[1]
        Wm, Wp = P[f"l{l}.Wm"], P[f"l{l}.Wp"]
        rmask = _replay_relu(lr.u, lr.u > 0,
                             None if hint is None else hint.relu[l], tau, stats,
                             f"layer {l}")
        du = dh * rmask
        G[f"l{l}.Wp"] = du.T @ lr.a
        G[f"l{l}.bp"] = du.sum(0)
        da = du @ Wp
        dh_prev = da[:, :F].copy()
        dA = (da[:, F:F + 4 * H] + rec.sp[:, None] * da[:, F + 4 * H:F + 8 * H]
              + rec.sm[:, None] * da[:, F + 8 * H:F + 12 * H])
        seg = lambda i: lr.m[csr.csr_eid[csr.rowptr[i]:csr.rowptr[i + 1]]]
        m_rms = _rms(lr.m)
        amin = _replay_arg(seg, lr.argmin, None if hint is None else hint.argmin[l],
                           tau, m_rms, stats, f"layer {l}", "argmin")
        amax = _replay_arg(seg, lr.argmax, None if hint is None else hint.argmax[l],
                           tau, m_rms, stats, f"layer {l}", "argmax")
        dm = np.zeros_like(lr.m)
        cols = np.arange(H)
        for i in range(N):
            lo, hi = int(csr.rowptr[i]), int(csr.rowptr[i + 1])
            d = hi - lo
            if d == 0:
                continue
            eids = csr.csr_eid[lo:hi]
            mu = lr.A[i, 0:H]
            sig = lr.A[i, 3 * H:4 * H]
            dm[eids] += dA[i, 0:H] / d
            dm[eids[amin[i]], cols] += dA[i, H:2 * H]
            dm[eids[amax[i]], cols] += dA[i, 2 * H:3 * H]
            dm[eids] += dA[i, 3 * H:4 * H] * (lr.m[eids] - mu) / (d * sig)
        G[f"l{l}.Wm"] = dm.T @ lr.z
        G[f"l{l}.bm"] = dm.sum(0)
        dz = dm @ Wm
        np.add.at(dh_prev, dst, dz[:, 0:F])
        np.add.at(dh_prev, src, dz[:, F:2 * F])
        dh = dh_prev
    return dh


# --------------------------------------------------------------------------
# AdamW (decoupled weight decay), t >= 1
# --------------------------------------------------------------------------

def adamw(theta, grad, m, v, t: int, lr: float = 1e-3, beta1: float = 0.9,
          beta2: float = 0.999, eps: float = 1e-8, weight_decay: float = 0.0):
    """One AdamW step; returns (theta', m', v') in float64."""
    theta = np.asarray(theta, np.float64) * (1.0 - lr * weight_decay)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
