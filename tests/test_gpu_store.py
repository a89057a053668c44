"""Packed graph store read on the GPU: batches handed out by the library's
reader give the same predictions, loss and training trajectory as the same
batches copied from host memory."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2207_11333_amd import graphstore as gs
from paper_2207_11333_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _model(w):
    from paper_2207_11333_amd import hgnn
    m = hgnn.Model(w.num_layers, w.hidden, 9, w.edge_feat, 4, w.precision, w.recompute, w.delta)
    m.set_params(w.params())
    return m


def test_store_batches_match_host_batches(tmp_path):
    from paper_2207_11333_amd import hgnn
    w = synth.WORKLOADS["c0_small_fp32"]
    bs = [synth.make_batch(100 + i, 16 + 3 * i, 5, 30, w.edge_feat) for i in range(5)]
    path = str(tmp_path / "c0.bin")
    gs.write_store(path, bs, edge_feat=w.edge_feat)
    store = hgnn.GraphStore(path, io_threads=2, host_slots=3)
    assert store.info["num_batches"] == 5
    ma, mb = _model(w), _model(w)
    for step in range(12):                       # more than two passes over the file
        sb = store.next()
        assert sb.index == step % 5
        ref = bs[sb.index]
        pa = torch.empty(ref.num_graphs, device="cuda")
        pb = torch.empty(ref.num_graphs, device="cuda")
        la = torch.empty(1, device="cuda")
        lb = torch.empty(1, device="cuda")
        ma.forward(sb, pa, la)
        mb.forward(hgnn.DeviceBatch.from_host(ref), pb, lb)
        ma.backward(); mb.backward()
        ma.adam_step(); mb.adam_step()
        torch.cuda.synchronize()
        assert torch.equal(pa, pb), f"step {step}"
        assert torch.equal(la, lb)
    assert torch.equal(ma.params(), mb.params())
    say(f"store: 12 steps over 5 batches equal to host-copied batches; final loss {la.item():.4f}")
    store.close()
    ma.close(); mb.close()


def test_store_open_errors(tmp_path):
    from paper_2207_11333_amd import hgnn
    with pytest.raises(hgnn.HgnnError):
        hgnn.GraphStore(str(tmp_path / "missing.bin"))
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"HGNNSTR1" + bytes(56))
    with pytest.raises(hgnn.HgnnError):
        hgnn.GraphStore(str(bad))
