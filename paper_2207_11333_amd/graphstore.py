"""Writer (and a plain NumPy reader) of the packed graph store.

The store keeps batches of molecular graphs in the layout of the paper's
Table 1 -- x [N, F], edge_index [2, E], edge_attr [E, Fe], y [B], plus the
graph offsets graph_ptr [B+1] -- one contiguous record per batch, so the
library's reader (hgnn_store_open / hgnn_store_next) moves a whole batch with
one read and one host-to-device copy.  Section 3.3 of the paper motivates
this: per-graph files and per-graph unpickling dominated its loading time.

File (little endian): a 64-byte header, an index of one entry per batch, and
the records, each starting at a multiple of 4096 bytes with its sections
256-byte aligned (the layout is restated in include/hgnn.h).
"""
from __future__ import annotations

import struct
from typing import Iterable, List

import numpy as np

from .synth import Batch

MAGIC = b"HGNNSTR1"
VERSION = 1
HEADER = struct.Struct("<8s8I3Q")          # magic, version, nb, F, Fe, has_y, 3 reserved, idx, 2 reserved
ENTRY = struct.Struct("<QQ4i")             # offset, bytes, B, N, E, reserved
assert HEADER.size == 64 and ENTRY.size == 32


def _a256(v: int) -> int:
    return (v + 255) & ~255


def sections(B: int, N: int, E: int, F: int, Fe: int, has_y: bool) -> dict:
    """Byte offsets of the sections inside one record, and its size."""
    gp = 0
    x = _a256(4 * (B + 1))
    ei = x + _a256(4 * N * F)
    ea = ei + _a256(8 * E)
    y = ea + _a256(4 * E * Fe)
    end = y + (_a256(4 * B) if has_y else 0)
    return {"gp": gp, "x": x, "ei": ei, "ea": ea, "y": y, "end": end}


def write_store(path: str, batches: Iterable[Batch], node_feat: int = 9, edge_feat: int = 1,
                has_y: bool = True) -> List[dict]:
    """Write the batches; returns their index entries."""
    batches = list(batches)
    if not batches:
        raise ValueError("no batches")
    entries = []
    off = 4096 * ((HEADER.size + ENTRY.size * len(batches) + 4095) // 4096)
    for b in batches:
        if b.x.shape[1] != node_feat or b.edge_feat != edge_feat:
            raise ValueError("batch feature widths differ from the store's")
        sec = sections(b.num_graphs, b.num_nodes, b.num_edges, node_feat, edge_feat, has_y)
        entries.append({"offset": off, "bytes": sec["end"], "B": b.num_graphs,
                        "N": b.num_nodes, "E": b.num_edges})
        off += 4096 * ((sec["end"] + 4095) // 4096)
    index_offset = HEADER.size
    with open(path, "wb") as f:
        f.write(HEADER.pack(MAGIC, VERSION, len(batches), node_feat, edge_feat, int(has_y),
                            0, 0, 0, index_offset, 0, 0))
        for e in entries:
            f.write(ENTRY.pack(e["offset"], e["bytes"], e["B"], e["N"], e["E"], 0))
        for b, e in zip(batches, entries):
            sec = sections(e["B"], e["N"], e["E"], node_feat, edge_feat, has_y)
            rec = bytearray(sec["end"])
            parts = [("gp", np.ascontiguousarray(b.graph_ptr, np.int32)),
                     ("x", np.ascontiguousarray(b.x, np.float32)),
                     ("ei", np.ascontiguousarray(b.edge_index, np.int32))]
            if edge_feat:
                parts.append(("ea", np.ascontiguousarray(b.edge_attr, np.float32)))
            if has_y:
                parts.append(("y", np.ascontiguousarray(b.y, np.float32)))
            for key, arr in parts:
                raw = arr.tobytes()
                rec[sec[key]:sec[key] + len(raw)] = raw
            f.seek(e["offset"])
            f.write(rec)
    return entries


def read_batch(path: str, i: int) -> Batch:
    """Batch i of a store, read back with NumPy (reference reader)."""
    with open(path, "rb") as f:
        h = HEADER.unpack(f.read(HEADER.size))
        if h[0] != MAGIC or h[1] != VERSION:
            raise ValueError("not a version-1 graph store")
        nb, F, Fe, has_y, idx = h[2], h[3], h[4], bool(h[5]), h[9]
        if not 0 <= i < nb:
            raise IndexError(i)
        f.seek(idx + ENTRY.size * i)
        off, nbytes, B, N, E, _ = ENTRY.unpack(f.read(ENTRY.size))
        f.seek(off)
        rec = f.read(nbytes)
    sec = sections(B, N, E, F, Fe, has_y)

    def arr(key, dtype, count, shape):
        return np.frombuffer(rec, dtype, count, sec[key]).reshape(shape).copy()

    return Batch(arr("gp", np.int32, B + 1, (B + 1,)), arr("x", np.float32, N * F, (N, F)),
                 arr("ei", np.int32, 2 * E, (2, E)),
                 arr("ea", np.float32, E * Fe, (E, Fe)) if Fe else None,
                 arr("y", np.float32, B, (B,)) if has_y else np.zeros(B, np.float32))
