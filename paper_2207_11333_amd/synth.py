"""Seeded synthetic molecule-shaped batches and seeded weight initialisation.

This module is the only code shared by the FP64 oracle's tests and the HIP
path.  It draws random numbers and lays them out in the graph schema of the
paper's Table 1 (``x`` [#nodes, #node features], ``edge_index`` [2, #edges],
``edge_attr`` [#edges, #edge features], one graph-level target per graph).  It
contains none of the method's arithmetic: no message, aggregation, scaler,
pooling, loss or gradient is computed here.

The datasets of the paper (PCQM4Mv2 and AISD HOMO-LUMO, Section 5.1, Table 2)
are not available; these batches stand in for them.  Their shape follows
Table 2 (about 29-52 atoms per molecule, about two directed edges per atom) and
the bounded valence of molecules (degree at most 4).

Recipe, per graph, in this RNG order (``numpy.random.Generator(PCG64(seed))``):
  1. node count n ~ integers(lo, hi + 1)
  2. atom type ~ integers(0, 5) per node, one-hot into 5 floats, then 4
     scalars ~ N(0, 1) per node: x has 9 floats per node
  3. spanning tree: for v = 1..n-1 the parent is uniform over the earlier
     nodes whose degree is still below 4
  4. round(0.1 * (n - 1)) extra bonds, each a uniform non-adjacent pair with
     both degrees below 4 (skipped when no such pair is left)
  5. every bond u-v is stored as u->v then v->u, in insertion order; one bond
     length ~ U(0.9, 1.6) is drawn per bond and shared by both directions
     (only when edge features are requested)
  6. target ~ N(5, 1.5)
Graphs are concatenated; node ids in ``edge_index`` are global.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

NODE_FEAT = 9
MAX_VALENCE = 4


@dataclasses.dataclass
class Batch:
    """A packed batch of graphs in the paper's Table 1 layout (host arrays)."""
    graph_ptr: np.ndarray          # int32 [B+1]; graph b owns nodes [ptr[b], ptr[b+1])
    x: np.ndarray                  # float32 [N, 9]
    edge_index: np.ndarray         # int32 [2, E]; row 0 source, row 1 destination
    edge_attr: Optional[np.ndarray]  # float32 [E, Fe] or None when Fe == 0
    y: np.ndarray                  # float32 [B]

    @property
    def num_graphs(self) -> int:
        return int(self.graph_ptr.shape[0] - 1)

    @property
    def num_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def num_edges(self) -> int:
        return int(self.edge_index.shape[1])

    @property
    def edge_feat(self) -> int:
        return 0 if self.edge_attr is None else int(self.edge_attr.shape[1])


def _one_graph(rng: np.random.Generator, lo: int, hi: int, edge_feat: int):
    n = int(rng.integers(lo, hi + 1))
    atom = rng.integers(0, 5, size=n)
    x = np.zeros((n, NODE_FEAT), dtype=np.float64)
    x[np.arange(n), atom] = 1.0
    x[:, 5:] = rng.standard_normal((n, 4))
    deg = np.zeros(n, dtype=np.int64)
    adj = np.zeros((n, n), dtype=bool)
    bonds: List[tuple] = []
    for v in range(1, n):
        cand = np.flatnonzero(deg[:v] < MAX_VALENCE)
        u = int(cand[rng.integers(0, cand.shape[0])])
        bonds.append((u, v))
        deg[u] += 1
        deg[v] += 1
        adj[u, v] = adj[v, u] = True
    extra = int(round(0.1 * (n - 1)))
    for _ in range(extra):
        ok = deg < MAX_VALENCE
        mask = np.triu(~adj & ok[:, None] & ok[None, :], 1)
        pairs = np.argwhere(mask)
        if pairs.shape[0] == 0:
            continue
        u, v = (int(t) for t in pairs[rng.integers(0, pairs.shape[0])])
        bonds.append((u, v))
        deg[u] += 1
        deg[v] += 1
        adj[u, v] = adj[v, u] = True
    src = np.empty(2 * len(bonds), dtype=np.int64)
    dst = np.empty(2 * len(bonds), dtype=np.int64)
    for j, (u, v) in enumerate(bonds):
        src[2 * j], dst[2 * j] = u, v
        src[2 * j + 1], dst[2 * j + 1] = v, u
    attr = None
    if edge_feat > 0:
        length = rng.uniform(0.9, 1.6, size=(len(bonds), edge_feat))
        attr = np.repeat(length, 2, axis=0)
    target = float(rng.normal(5.0, 1.5))
    return x, src, dst, attr, target


def make_batch(seed: int, num_graphs: int, n_lo: int, n_hi: int,
               edge_feat: int) -> Batch:
    """Draw ``num_graphs`` molecule-shaped graphs and pack them (see module doc)."""
    if num_graphs < 0 or n_lo < 1 or n_hi < n_lo or edge_feat < 0:
        raise ValueError("bad generator arguments")
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, srcs, dsts, attrs, ys = [], [], [], [], []
    ptr = [0]
    for _ in range(num_graphs):
        x, s, d, a, t = _one_graph(rng, n_lo, n_hi, edge_feat)
        off = ptr[-1]
        xs.append(x)
        srcs.append(s + off)
        dsts.append(d + off)
        if a is not None:
            attrs.append(a)
        ys.append(t)
        ptr.append(off + x.shape[0])
    n_tot = ptr[-1]
    x = np.concatenate(xs, 0) if xs else np.zeros((0, NODE_FEAT))
    src = np.concatenate(srcs) if srcs else np.zeros(0, np.int64)
    dst = np.concatenate(dsts) if dsts else np.zeros(0, np.int64)
    edge_attr = None
    if edge_feat > 0:
        edge_attr = (np.concatenate(attrs, 0) if attrs
                     else np.zeros((0, edge_feat))).astype(np.float32)
    assert n_tot < 2**31 and src.shape[0] < 2**31
    return Batch(graph_ptr=np.asarray(ptr, dtype=np.int32),
                 x=x.astype(np.float32),
                 edge_index=np.stack([src, dst]).astype(np.int32),
                 edge_attr=edge_attr,
                 y=np.asarray(ys, dtype=np.float32))


def concat_batches(parts: Sequence[Batch]) -> Batch:
    """Concatenate packed batches graph-wise (node ids are re-offset)."""
    ptr = [0]
    xs, eis, eas, ys = [], [], [], []
    for p in parts:
        off = ptr[-1]
        ptr.extend((p.graph_ptr[1:].astype(np.int64) + off).tolist())
        xs.append(p.x)
        eis.append(p.edge_index.astype(np.int64) + off)
        if p.edge_attr is not None:
            eas.append(p.edge_attr)
        ys.append(p.y)
    fe = parts[0].edge_feat if parts else 0
    return Batch(graph_ptr=np.asarray(ptr, dtype=np.int32),
                 x=np.concatenate(xs, 0).astype(np.float32),
                 edge_index=np.concatenate(eis, 1).astype(np.int32),
                 edge_attr=(np.concatenate(eas, 0).astype(np.float32) if fe else None),
                 y=np.concatenate(ys).astype(np.float32))


def select_graphs(b: Batch, graphs: Sequence[int]) -> Batch:
    """Extract the listed graphs (in the given order) as a new packed batch."""
    parts = []
    src, dst = b.edge_index
    for g in graphs:
        lo, hi = int(b.graph_ptr[g]), int(b.graph_ptr[g + 1])
        sel = (dst >= lo) & (dst < hi)
        parts.append(Batch(
            graph_ptr=np.asarray([0, hi - lo], np.int32),
            x=b.x[lo:hi],
            edge_index=np.stack([src[sel] - lo, dst[sel] - lo]).astype(np.int32),
            edge_attr=None if b.edge_attr is None else b.edge_attr[sel],
            y=b.y[g:g + 1]))
    return concat_batches(parts)


# ---------------------------------------------------------------------------
# Model shapes and the parameter packing order (interchange/checkpoint order).
# Every matrix is row-major [out, in].  Per layer l (input width F_l, F_1 = 9,
# F_l = H afterwards): W^m [H, 2F+Fe], b^m [H], W^p [H, F+12H], b^p [H];
# then the head W1 [H, H], b1 [H], w2 [1, H], b2 [1].
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ModelShape:
    num_layers: int
    hidden: int
    node_feat: int = NODE_FEAT
    edge_feat: int = 1

    def layer_in(self, l: int) -> int:
        return self.node_feat if l == 0 else self.hidden

    def tensor_shapes(self):
        """[(name, shape)] in packing order."""
        H, Fe = self.hidden, self.edge_feat
        out = []
        for l in range(self.num_layers):
            F = self.layer_in(l)
            out += [(f"l{l}.Wm", (H, 2 * F + Fe)), (f"l{l}.bm", (H,)),
                    (f"l{l}.Wp", (H, F + 12 * H)), (f"l{l}.bp", (H,))]
        out += [("W1", (H, H)), ("b1", (H,)), ("w2", (1, H)), ("b2", (1,))]
        return out

    def num_params(self) -> int:
        return int(sum(int(np.prod(s)) for _, s in self.tensor_shapes()))

    def offsets(self):
        """{name: (offset, shape)} into the packed vector."""
        off, res = 0, {}
        for name, shp in self.tensor_shapes():
            res[name] = (off, shp)
            off += int(np.prod(shp))
        return res


def init_params(shape: ModelShape, seed: int) -> np.ndarray:
    """Seeded Xavier-uniform weights, U(+-0.1) biases, drawn in packing order.

    Returns the packed float32 vector handed identically to the oracle and to
    the device context.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    chunks = []
    for name, shp in shape.tensor_shapes():
        if len(shp) == 2:
            a = np.sqrt(6.0 / (shp[0] + shp[1]))
            chunks.append(rng.uniform(-a, a, size=shp).ravel())
        else:
            chunks.append(rng.uniform(-0.1, 0.1, size=shp))
    return np.concatenate(chunks).astype(np.float32)


_SM_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64_at(seed: int, j: np.ndarray) -> np.ndarray:
    """Output j (0-based) of SplitMix64 started from `seed` (Steele, Lea and
    Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
    mix(seed + (j + 1) * gamma), as uint64 (numpy wraps modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (np.asarray(j, np.uint64) + np.uint64(1)) * np.uint64(_SM_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def counter_init_params(tensor_shapes, seed: int) -> np.ndarray:
    """The device-side seeded initialisation, written out on the host: element
    j of the packed vector is bound * k * 2^-23 (FP32, one rounding) with
    k = (z >> 40) - 2^23 and z = splitmix64_at(seed, j); bound is
    sqrt(6 / (rows + cols)) for a weight [rows, cols] (Xavier-uniform) and 0.1
    for a bias (1-D shape)."""
    chunks, off = [], 0
    for _, shp in tensor_shapes:
        n = int(np.prod(shp))
        j = np.arange(off, off + n, dtype=np.uint64)
        k = (splitmix64_at(seed, j) >> np.uint64(40)).astype(np.int64) - (1 << 23)
        bound = np.float32(np.sqrt(6.0 / (shp[0] + shp[1]))) if len(shp) == 2 else np.float32(0.1)
        chunks.append(bound * (k.astype(np.float32) * np.float32(2.0 ** -23)))
        off += n
    return np.concatenate(chunks).astype(np.float32)


def gc_tensor_shapes(kind: str, num_layers: int, hidden: int, node_feat: int = NODE_FEAT,
                     edge_feat: int = 1, graph_heads: int = 1, node_heads: int = 0):
    """[(name, shape)] of a GraphSAGE ("sage") or CGCNN ("cgcnn") model in
    packing order: the GC stack, then the graph heads, then the node heads."""
    H, Fe = hidden, edge_feat
    out = []
    if kind == "sage":
        for l in range(num_layers):
            F = node_feat if l == 0 else H
            out += [(f"l{l}.W", (H, 2 * F)), (f"l{l}.b", (H,))]
    elif kind == "cgcnn":
        out += [("emb.W", (H, node_feat)), ("emb.b", (H,))]
        for l in range(num_layers):
            out += [(f"l{l}.W", (2 * H, 2 * H + Fe)), (f"l{l}.b", (2 * H,))]
    else:
        raise ValueError(f"unknown layer kind {kind!r}")
    for t in range(graph_heads + node_heads):
        out += [(f"h{t}.W1", (H, H)), (f"h{t}.b1", (H,)), (f"h{t}.w2", (1, H)),
                (f"h{t}.b2", (1,))]
    return out


def init_gc_params(kind: str, num_layers: int, hidden: int, seed: int,
                   node_feat: int = NODE_FEAT, edge_feat: int = 1, graph_heads: int = 1,
                   node_heads: int = 0) -> np.ndarray:
    """Seeded Xavier-uniform matrices, U(+-0.1) biases, in packing order (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    chunks = []
    for _, shp in gc_tensor_shapes(kind, num_layers, hidden, node_feat, edge_feat,
                                   graph_heads, node_heads):
        if len(shp) == 2:
            a = np.sqrt(6.0 / (shp[0] + shp[1]))
            chunks.append(rng.uniform(-a, a, size=shp).ravel())
        else:
            chunks.append(rng.uniform(-0.1, 0.1, size=shp))
    return np.concatenate(chunks).astype(np.float32)


# ---------------------------------------------------------------------------
# Workload presets.  ``delta`` is the PNA degree normaliser: the mean of
# ln(d+1) over every node of 10,000 generator graphs (seed 3000 + c), written
# out by oracle/calibrate_delta.py and pasted here as a model constant.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    num_layers: int
    hidden: int
    num_graphs: int
    n_lo: int
    n_hi: int
    edge_feat: int
    precision: int        # 0 = FP32 linears, 1 = BF16 MFMA operands
    recompute: int
    data_seed: int
    weight_seed: int
    delta: float

    @property
    def shape(self) -> ModelShape:
        return ModelShape(self.num_layers, self.hidden, NODE_FEAT, self.edge_feat)

    def batch(self) -> Batch:
        return make_batch(self.data_seed, self.num_graphs, self.n_lo, self.n_hi,
                          self.edge_feat)

    def params(self) -> np.ndarray:
        return init_params(self.shape, self.weight_seed)


DELTA_C0 = 1.0666336621019612
DELTA_C1 = 1.0839407315514658
DELTA_C3 = 1.086156263580869

WORKLOADS = {
    "c0_small_fp32": Workload("c0_small_fp32", 3, 64, 64, 5, 30, 0, 0, 0,
                              1000, 2000, DELTA_C0),
    "c1_train_fp32": Workload("c1_train_fp32", 6, 128, 128, 10, 60, 1, 0, 0,
                              1001, 2001, DELTA_C1),
    "c2_train_bf16": Workload("c2_train_bf16", 6, 128, 128, 10, 60, 1, 1, 0,
                              1001, 2001, DELTA_C1),
    "c3_large_bf16": Workload("c3_large_bf16", 8, 256, 1024, 10, 70, 1, 1, 1,
                              1003, 2003, DELTA_C3),
}

SERVE_WORKLOAD = dict(num_layers=6, hidden=128, edge_feat=1, precision=1,
                      weight_seed=2004, delta=DELTA_C1, mol_lo=1, mol_hi=256,
                      n_lo=5, n_hi=70, request_seed=4000, arrival_seed=4004)


def make_request(rng: np.random.Generator, mol_lo: int, mol_hi: int, n_lo: int,
                 n_hi: int, edge_feat: int) -> Batch:
    """One serving request: a packed batch of 1..256 molecules (5-70 atoms)."""
    b = int(rng.integers(mol_lo, mol_hi + 1))
    return make_batch(int(rng.integers(0, 2**62)), b, n_lo, n_hi, edge_feat)
