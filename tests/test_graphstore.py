"""Packed graph store: the file writer and its NumPy reader (host only)."""
import os

import numpy as np
import pytest

from paper_2207_11333_amd import graphstore as gs
from paper_2207_11333_amd import synth


def _batches():
    return [synth.make_batch(seed, 3 + seed, 5, 12, 1) for seed in range(5)]


def test_round_trip_and_alignment(tmp_path):
    path = str(tmp_path / "s.bin")
    bs = _batches()
    entries = gs.write_store(path, bs)
    assert all(e["offset"] % 4096 == 0 for e in entries)
    for i, b in enumerate(bs):
        r = gs.read_batch(path, i)
        np.testing.assert_array_equal(r.graph_ptr, b.graph_ptr)
        np.testing.assert_array_equal(r.x, b.x)
        np.testing.assert_array_equal(r.edge_index, b.edge_index)
        np.testing.assert_array_equal(r.edge_attr, b.edge_attr)
        np.testing.assert_array_equal(r.y, b.y)
    sec = gs.sections(3, 40, 70, 9, 1, True)
    assert all(sec[k] % 256 == 0 for k in ("gp", "x", "ei", "ea", "y"))
    assert sec["end"] >= sec["y"] + 4 * 3


def test_without_edge_features(tmp_path):
    path = str(tmp_path / "s0.bin")
    b = synth.make_batch(7, 4, 5, 9, 0)
    gs.write_store(path, [b], edge_feat=0)
    r = gs.read_batch(path, 0)
    assert r.edge_attr is None
    np.testing.assert_array_equal(r.edge_index, b.edge_index)


def test_rejects_bad_files(tmp_path):
    path = str(tmp_path / "bad.bin")
    with open(path, "wb") as f:
        f.write(b"NOTASTOR" + bytes(56))
    with pytest.raises(ValueError):
        gs.read_batch(path, 0)
    with pytest.raises(ValueError):
        gs.write_store(str(tmp_path / "w.bin"), [synth.make_batch(1, 2, 5, 9, 1)], edge_feat=0)
    with pytest.raises(IndexError):
        p2 = str(tmp_path / "one.bin")
        gs.write_store(p2, [synth.make_batch(1, 2, 5, 9, 1)])
        gs.read_batch(p2, 1)
